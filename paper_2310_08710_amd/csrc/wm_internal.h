// wm_internal.h -- argument blocks shared by the kernels and the host API,
// the workspace layout and the launch entry points of wm_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/wm.h"

namespace wm {

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Road-edge points per chunk of the off-road scan.
constexpr int kEdgeChunk = 128;

// First point slot of scenario s in the compacted road-edge arrays: a whole
// number of chunks, at least P_s + kEdgeChunk slots before the next scenario's.
__host__ __device__ inline long edge_base(int rg_off_s, int s)
{
    return (long)kEdgeChunk * ((long)rg_off_s / kEdgeChunk + 2L * s);
}

// Compacted road edges in the workspace.  Scenario s owns the point slots
// from edge_base(rg_off[s], s): its valid road edges in index order, padded
// to whole chunks (two spare chunks at the end of the arrays let the scan
// prefetch past the last chunk).  `stream` holds chunk c
// of that range as x[128], y[128], qq[128] (qq = x^2 + y^2, rotated within
// groups of four, see qq_slot in wm_device.h; padding points have
// x = y = 0 and qq = +inf); `dir` and `idx` (scenario-local original index)
// are indexed by point.  `count` = edges per scenario, `qqmax` = their max qq.
// `box` holds, per 32 stream points (a block), the box (xmin, xmax, ymin,
// ymax) of its edge points, and `cbox` the same per chunk; blocks and chunks
// of a scenario start at box[base / 32] and cbox[base / 128].  A box without
// points is (+inf, -inf, +inf, -inf).
constexpr int kBoxPts = 32;
struct Edges {
    float *stream;
    float2 *dir;
    int32_t *idx;
    int32_t *count;
    float *qqmax;
    float4 *box;
    float4 *cbox;
};

struct StepArgs {
    const int32_t *obj_off;
    wm_state cur;
    wm_action act;
    wm_state log_next;
    wm_state next;
    float dt;
    float *log_div;
    uint8_t *infeasible;
};

struct OverlapArgs {
    const int32_t *obj_off;
    wm_state st;
    const int64_t *pair_off;
    float *margin;
    uint8_t *mask;
    uint8_t *collision;
    float *max_margin;
    int maxN;
    int U;
};

struct OffroadArgs {
    const int32_t *obj_off, *rg_off;
    wm_state st;
    Edges E;
    uint8_t *offroad;
    float *margin;
    int32_t *nearest;
    int G, CW;
};

struct RollArgs {
    int S, n, T, ckpt_every, maxN, G, CW;
    float dt;
    const int32_t *obj_off, *rg_off;
    wm_state init;
    wm_action act;
    wm_state log;
    int has_rg, has_ckpt, has_traj, want_loss;
    Edges E;
    wm_state ckpt, traj;
    wm_metrics met;
    float *lossp;
    const int32_t *uoff;
    const int2 *units;
    int32_t *counter;
    // IDM sim agents (has_idm): parameters, the object-major paths
    // [n][T+1] of (x, y, yaw, arc length) and the per-object agent flags
    int has_idm;
    wm_idm idm;
    const float4 *idmP;
    const uint8_t *idmA;
};

struct ObserveArgs {
    const int32_t *obj_off, *rg_off;
    wm_state st;            // row 0; row t (grid y) is st + t * n
    wm_roadgraph rg;
    const int32_t *ego;
    int E, k, maxN;
    int32_t *rg_idx;        // outputs of row t follow those of row t - 1
    float *rg_feat, *obj_feat;
    long n, S;              // state row stride (objects), scenarios
};

struct BackwardArgs {
    int S, n, T, K, maxN;
    int SB;          // steps per pair work-group (backward_block_steps)
    float dt;
    const int32_t *obj_off;
    wm_state init;
    wm_action act;
    wm_state log;
    wm_state ckpt;
    const float *dloss;
    float *grad_a, *grad_k;
    float *rec;      // [T][n][kRecFields] the reverse recursion's inputs per step and object
    float *part;     // [T][n][4] pair-term sums per step and controlled object
};

// The queue counter area (16 int32): [0] next unit, [1] units; from int32
// index kRollCounts, kRollCountN 64-bit work counts of the fused rollout's
// off-road scan (wm_rollout_scan_counts).
constexpr int kRollCounts = 4;
constexpr int kRollCountN = 3;

// Workspace rows of the adjoint's recursion inputs per step and object.
constexpr int kRecFields = 16;

// Workspace sections (byte offsets, each 256-aligned).
struct WsLayout {
    size_t ecount, stream, edir, eidx, qqmax, ebox, ecbox, uoff, units, lossp, counter, seg, idmP, idmA, total;
};

inline WsLayout ws_layout(int S, int n, int P, int T, int K)
{
    const size_t cap = (size_t)P + 2 * (size_t)S * kEdgeChunk + 2 * kEdgeChunk;
    WsLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    L.ecount = take(sizeof(int32_t) * (size_t)S);
    L.stream = take(sizeof(float) * 3 * cap);
    L.edir = take(sizeof(float) * 2 * cap);
    L.eidx = take(sizeof(int32_t) * cap);
    L.qqmax = take(sizeof(float) * (size_t)S);
    L.ebox = take(sizeof(float) * 4 * (cap / kBoxPts + 1));
    L.ecbox = take(sizeof(float) * 4 * (cap / kEdgeChunk + 1));
    L.uoff = take(sizeof(int32_t) * ((size_t)S + 1));
    L.units = take(sizeof(int32_t) * 2 * ((size_t)n + 1));
    L.lossp = take(sizeof(float) * ((size_t)n + 1));
    L.counter = take(sizeof(int32_t) * 16);
    L.seg = (T > 0 && K > 0) ? take(sizeof(float) * (kRecFields + 4) * (size_t)T * (size_t)n) : o;
    L.idmP = T > 0 ? take(sizeof(float) * 4 * (size_t)(T + 1) * (size_t)n) : o;
    L.idmA = T > 0 ? take((size_t)n + 1) : o;
    L.total = o;
    return L;
}

inline Edges ws_edges(unsigned char *ws, const WsLayout &L)
{
    return Edges{(float *)(ws + L.stream), (float2 *)(ws + L.edir), (int32_t *)(ws + L.eidx),
                 (int32_t *)(ws + L.ecount), (float *)(ws + L.qqmax), (float4 *)(ws + L.ebox),
                 (float4 *)(ws + L.ecbox)};
}

// Launchers (wm_kernels.hip).  They only enqueue; errors surface through
// hipGetLastError in the caller.
void launch_compact_edges(const wm_batch &b, const wm_roadgraph &rg, unsigned char *ws, const WsLayout &L,
                          hipStream_t st);
void launch_edge_boxes(const wm_batch &b, unsigned char *ws, const WsLayout &L, hipStream_t st);
void launch_build_units(const wm_batch &b, int U, const int32_t *ecount, unsigned char *ws, const WsLayout &L,
                        hipStream_t st);
void launch_dynamics(const wm_batch &b, const StepArgs &a, hipStream_t st);
void launch_reward(const wm_batch &b, const uint8_t *col, const uint8_t *off, float *reward, hipStream_t st);
void launch_delta_step(const wm_batch &b, const wm_state &cur, const wm_delta_action &act, const wm_state &log_next,
                       const wm_state &next, float dt, hipStream_t st);
void launch_delta_inverse(int n, const wm_state &cur, const wm_state &nxt, float *dx, float *dy, float *dyaw,
                          uint8_t *vout, hipStream_t st);
void launch_discretize(int n, const float *v, float lo, float scale, float step, int bins, int32_t *index,
                       float *snapped, hipStream_t st);
void launch_inverse(int n, const wm_state &cur, const wm_state &nxt, float dt, float *accel, float *curv,
                    uint8_t *vout, hipStream_t st);
void launch_overlap(const wm_batch &b, const OverlapArgs &a, hipStream_t st);
void launch_offroad(const wm_batch &b, const OffroadArgs &a, hipStream_t st);
size_t rollout_lds_bytes(int maxN, int G, int CW);
int rollout_grid(int G, int CW, int maxN, int n_units_bound);
void launch_rollout(const RollArgs &a, int grid, hipStream_t st);
void launch_idm_paths(int n, int T, const wm_state &log, const uint8_t *controlled, float4 *path, uint8_t *agent,
                      hipStream_t st);
void launch_loss_reduce(int S, const int32_t *uoff, const float *lossp, float *loss, hipStream_t st);
void launch_observe(const wm_batch &b, const ObserveArgs &a, int rows, hipStream_t st);
int backward_block_steps(int maxN, int K);
void launch_backward(const BackwardArgs &a, hipStream_t st);
// Device address of the current device's WM_NOALLOC_SCRATCH_BYTES scratch
// array (looked up on the first call per device).
hipError_t noalloc_scratch(unsigned char **out);

} // namespace wm
