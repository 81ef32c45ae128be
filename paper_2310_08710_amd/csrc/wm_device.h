// wm_device.h -- device building blocks of the simulator step for gfx950.
//
// Everything here is float32 and written with explicit fused multiply-adds
// (the library is compiled with -ffp-contract=off), so a quantity recomputed
// by a second kernel is bit-identical to the first computation.  That matters
// for the off-road rescan (argmin recovery) and for the adjoint's segment
// recomputation.
#pragma once

#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

#include "../../include/wm.h"
#include "wm_internal.h"

namespace wm {

constexpr int kChunk = kEdgeChunk;    // road-edge points per chunk of the off-road scan
constexpr float kNoValue = -FLT_MAX;  // margin with no defined value
constexpr float kSoftScale = 0.1f;    // soft-overlap scale of the training loss [m]

// Scenario-major packed state kept in LDS by the fused kernels.
struct ObjLds {
    float *x, *y, *yaw, *vx, *vy, *len, *wid, *c, *s;
    uint8_t *valid, *ctrl, *infeas;
};

// ---------------------------------------------------------------------------
// Bicycle forward dynamics (App. A.1, forward dynamics equation).
//   v = |(vx, vy)|; x' = x + vx dt + a cos(yaw) dt^2/2; y' likewise with sin;
//   yaw' = yaw + kappa (v dt + a dt^2/2); v' = v + a dt; (vx', vy') = v'(cos, sin)(yaw')
// ---------------------------------------------------------------------------
// The same step, also returning the sine and cosine of the yaw before (s, c)
// and after (ns, nc) it, which the adjoint's factors reuse.
__device__ __forceinline__ void bicycle_forward_sc(float &x, float &y, float &yaw, float &vx, float &vy,
                                                   float a, float k, float dt, float &s, float &c, float &ns,
                                                   float &nc)
{
    const float hdt2 = 0.5f * dt * dt;
    const float v = sqrtf(__builtin_fmaf(vy, vy, vx * vx));
    sincosf(yaw, &s, &c);
    const float ahdt2 = a * hdt2;
    const float nx = x + __builtin_fmaf(vx, dt, ahdt2 * c);
    const float ny = y + __builtin_fmaf(vy, dt, ahdt2 * s);
    const float dist = __builtin_fmaf(v, dt, ahdt2);
    const float nyaw = __builtin_fmaf(k, dist, yaw);
    const float nv = __builtin_fmaf(a, dt, v);
    sincosf(nyaw, &ns, &nc);
    x = nx;
    y = ny;
    yaw = nyaw;
    vx = nv * nc;
    vy = nv * ns;
}

__device__ __forceinline__ void bicycle_forward(float &x, float &y, float &yaw, float &vx, float &vy,
                                                float a, float k, float dt)
{
    const float hdt2 = 0.5f * dt * dt;
    const float v = sqrtf(__builtin_fmaf(vy, vy, vx * vx));
    float s, c;
    sincosf(yaw, &s, &c);
    const float ahdt2 = a * hdt2;
    const float nx = x + __builtin_fmaf(vx, dt, ahdt2 * c);
    const float ny = y + __builtin_fmaf(vy, dt, ahdt2 * s);
    const float dist = __builtin_fmaf(v, dt, ahdt2);
    const float nyaw = __builtin_fmaf(k, dist, yaw);
    const float nv = __builtin_fmaf(a, dt, v);
    float ns, nc;
    sincosf(nyaw, &ns, &nc);
    x = nx;
    y = ny;
    yaw = nyaw;
    vx = nv * nc;
    vy = nv * ns;
}

// wrap(a) = a - 2 pi floor((a + pi) / (2 pi)), in [-pi, pi)
__device__ __forceinline__ float wrap_angle(float a)
{
    const float two_pi = 6.28318530717958647692f;
    float r = a - two_pi * floorf((a + 3.14159265358979323846f) * (1.0f / two_pi));
    if (r >= 3.14159265358979323846f)
        r -= two_pi;
    if (r < -3.14159265358979323846f)
        r += two_pi;
    return r;
}

// Bicycle inverse kinematics (App. A.1, inverse kinematics equation) of one
// transition: a = (|v'| - |v|) / dt, kappa = wrap(atan2(vy', vx') - yaw) / D with
// D = |v| dt + a dt^2 / 2 (kappa = 0 when |D| < 1e-6 m).
__device__ __forceinline__ void inverse_kinematics(float vx, float vy, float yaw, float nvx, float nvy, float dt,
                                                   float &a, float &k)
{
    const float v = sqrtf(__builtin_fmaf(vy, vy, vx * vx));
    const float nv = sqrtf(__builtin_fmaf(nvy, nvy, nvx * nvx));
    a = (nv - v) / dt;
    const float dist = __builtin_fmaf(v, dt, 0.5f * a * dt * dt);
    k = fabsf(dist) < 1e-6f ? 0.f : wrap_angle(atan2f(nvy, nvx) - yaw) / dist;
}

// Kinematic infeasibility of a transition (Sec. 3.4): |a| > 6 or |kappa| > 0.3.
__device__ __forceinline__ uint8_t infeasible_transition(float vx, float vy, float yaw, float nvx, float nvy,
                                                         float dt)
{
    float a, k;
    inverse_kinematics(vx, vy, yaw, nvx, nvy, dt, a, k);
    return (uint8_t)(fabsf(a) > 6.f || fabsf(k) > 0.3f);
}

// ---------------------------------------------------------------------------
// Separating-axis overlap margin of two boxes (Sec. 3.4 Collision), with the
// unit heading (c, s) and half extents precomputed.  Axis order u_a, w_a,
// u_b, w_b; g = r_a + r_b - |d . axis|; margin = min g.  Callers pass the box
// with the lower index as `a` so that m_ij and m_ji are the same bits.
// ---------------------------------------------------------------------------
struct Box {
    float x, y, c, s, hl, hw;
};

__device__ __forceinline__ float sat_margin(const Box &a, const Box &b)
{
    const float dx = b.x - a.x, dy = b.y - a.y;
    const float C = fabsf(__builtin_fmaf(a.c, b.c, a.s * b.s));   // |cos(yaw_b - yaw_a)|
    const float S = fabsf(__builtin_fmaf(a.c, b.s, -(a.s * b.c))); // |sin(yaw_b - yaw_a)|
    const float g1 = a.hl + __builtin_fmaf(b.hl, C, b.hw * S) - fabsf(__builtin_fmaf(dx, a.c, dy * a.s));
    const float g2 = a.hw + __builtin_fmaf(b.hl, S, b.hw * C) - fabsf(__builtin_fmaf(dy, a.c, -(dx * a.s)));
    const float g3 = b.hl + __builtin_fmaf(a.hl, C, a.hw * S) - fabsf(__builtin_fmaf(dx, b.c, dy * b.s));
    const float g4 = b.hw + __builtin_fmaf(a.hl, S, a.hw * C) - fabsf(__builtin_fmaf(dy, b.c, -(dx * b.s)));
    return fminf(fminf(g1, g2), fminf(g3, g4));
}

// sat_margin(a, b) when a_first, else sat_margin(b, a), in one evaluation:
// swapping the boxes negates the offsets exactly and commutes the operands
// of every other product, so the two orders differ only in the rounding of
// |sin(yaw_b - yaw_a)|; the four gaps swap places, and the minimum of the
// same four values is taken.
__device__ __forceinline__ float sat_margin_ordered(const Box &a, const Box &b, bool a_first)
{
    const float dx = b.x - a.x, dy = b.y - a.y;
    const float C = fabsf(__builtin_fmaf(a.c, b.c, a.s * b.s));
    const float S = a_first ? fabsf(__builtin_fmaf(a.c, b.s, -(a.s * b.c))) : fabsf(__builtin_fmaf(b.c, a.s, -(b.s * a.c)));
    const float g1 = a.hl + __builtin_fmaf(b.hl, C, b.hw * S) - fabsf(__builtin_fmaf(dx, a.c, dy * a.s));
    const float g2 = a.hw + __builtin_fmaf(b.hl, S, b.hw * C) - fabsf(__builtin_fmaf(dy, a.c, -(dx * a.s)));
    const float g3 = b.hl + __builtin_fmaf(a.hl, C, a.hw * S) - fabsf(__builtin_fmaf(dx, b.c, dy * b.s));
    const float g4 = b.hw + __builtin_fmaf(a.hl, S, a.hw * C) - fabsf(__builtin_fmaf(dy, b.c, -(dx * b.s)));
    return fminf(fminf(g1, g2), fminf(g3, g4));
}

// ---------------------------------------------------------------------------
// IDM sim agents (Sec. 3.5; intelligent driver model).  An agent's path is
// its logged positions, rows 0..T of the log window, with cumulative arc
// lengths L (time-major [T+1][n] like the logs).
// ---------------------------------------------------------------------------

// An IDM agent's path, object-major: row k of object g is path[g * (T + 1)
// + k] = (x, y, yaw, L) of its logged state k, L the cumulative arc length.
// Pose at arc length s: linear between the rows k-1 and k around the first k
// with L_k > s (yaw along the shorter arc between the logged yaws), or row
// T's pose when there is no such row.  One path is 16 (T + 1) contiguous
// bytes, so the search and the interpolation stay in a few cache lines.

// Index lo of the first path point 1..T whose arc length w(k) exceeds s
// (T + 1: none); w non-decreasing.
template <class Wf>
__device__ __forceinline__ int idm_segment(Wf w, int T, float s)
{
    int lo = 1, hi = T + 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (w(mid) > s)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// idm_segment of arc lengths w(k) = path[k].w for an s whose segment is
// known to be at least lo0 (every row k < lo0 has w(k) <= s, e.g. the
// segment of an earlier, smaller arc length): the next four rows are loaded
// at once, the rest searched by bisection.  The same index as idm_segment.
__device__ __forceinline__ int idm_segment_from(const float4 *__restrict__ path, int T, float s, int lo0)
{
    lo0 = max(lo0, 1);
    float w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        w[j] = path[min(lo0 + j, T)].w;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (lo0 + j <= T && w[j] > s)
            return lo0 + j;
    int lo = min(lo0 + 4, T + 1), hi = T + 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (path[mid].w > s)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// The pose at arc length s given its segment lo (idm_segment): linear
// between path points lo - 1 and lo, the last point past the end.
__device__ __forceinline__ void idm_interp(const float4 *__restrict__ path, int T, int lo, float s, float &x, float &y,
                                           float &yaw)
{
    if (lo > T) {
        const float4 r = path[T];
        x = r.x;
        y = r.y;
        yaw = r.z;
        return;
    }
    const float4 a = path[lo - 1], b = path[lo];
    const float lam = (s - a.w) / (b.w - a.w);
    x = __builtin_fmaf(lam, b.x - a.x, a.x);
    y = __builtin_fmaf(lam, b.y - a.y, a.y);
    yaw = __builtin_fmaf(lam, wrap_angle(b.z - a.z), a.z);
}

// IDM acceleration for speed v; `lead` selects the interaction term with gap
// `gap` and lead speed vl (along the agent's yaw).
__device__ __forceinline__ float idm_accel(const wm_idm &p, float v, bool lead, float gap, float vl)
{
    float a = p.max_accel * (1.0f - powf(v / p.desired_speed, p.exponent));
    if (lead) {
        const float ss =
            p.min_gap + fmaxf(0.0f, v * p.time_headway + v * (v - vl) / (2.0f * sqrtf(p.max_accel * p.comfort_decel)));
        const float q = ss / gap;
        a = gap > 0.0f ? a - p.max_accel * (q * q) : -p.max_brake;
    }
    return fminf(fmaxf(a, -p.max_brake), p.max_accel);
}

// Margin of the separating-axis test (the same value as sat_margin) and its
// gradient with respect to (x, y, yaw) of box a (of_b false) or box b (of_b
// true), through the arg-min axis (lowest axis index on ties), sgn(0) = +1.
__device__ __forceinline__ float sat_margin_grad_one(const Box &a, const Box &b, bool of_b, float &gx, float &gy,
                                                     float &gt)
{
    const float dx = b.x - a.x, dy = b.y - a.y;
    const float cd = __builtin_fmaf(a.c, b.c, a.s * b.s);    // cos(delta), delta = yaw_b - yaw_a
    const float sd = __builtin_fmaf(a.c, b.s, -(a.s * b.c)); // sin(delta)
    const float C = fabsf(cd), S = fabsf(sd);
    const float dC = -(cd >= 0.f ? 1.f : -1.f) * sd;
    const float dS = (sd >= 0.f ? 1.f : -1.f) * cd;
    const float pua = __builtin_fmaf(dx, a.c, dy * a.s), pwa = __builtin_fmaf(dy, a.c, -(dx * a.s));
    const float pub = __builtin_fmaf(dx, b.c, dy * b.s), pwb = __builtin_fmaf(dy, b.c, -(dx * b.s));
    const float g0 = a.hl + __builtin_fmaf(b.hl, C, b.hw * S) - fabsf(pua);
    const float g1 = a.hw + __builtin_fmaf(b.hl, S, b.hw * C) - fabsf(pwa);
    const float g2 = b.hl + __builtin_fmaf(a.hl, C, a.hw * S) - fabsf(pub);
    const float g3 = b.hw + __builtin_fmaf(a.hl, S, a.hw * C) - fabsf(pwb);
    // arg-min with selects (lowest index on ties)
    const bool k1 = g1 < g0;
    float m = k1 ? g1 : g0;
    const bool k2 = g2 < m;
    m = k2 ? g2 : m;
    const bool k3 = g3 < m;
    m = k3 ? g3 : m;
    const int k = k3 ? 3 : (k2 ? 2 : (k1 ? 1 : 0));
    const bool on_a = k < 2, odd = (k & 1) != 0;
    // axis (ax, ay), projection p of the offset on it, d(radius)/d(delta) rd,
    // and d(p)/d(own yaw) of the box whose axis it is
    const float bc = on_a ? a.c : b.c, bs = on_a ? a.s : b.s;
    const float ax = odd ? -bs : bc, ay = odd ? bc : bs;
    const float p = on_a ? (odd ? pwa : pua) : (odd ? pwb : pub);
    const float hl = on_a ? b.hl : a.hl, hw = on_a ? b.hw : a.hw;
    const float rd = odd ? __builtin_fmaf(hl, dS, hw * dC) : __builtin_fmaf(hl, dC, hw * dS);
    const float dp = on_a ? (odd ? -pua : pwa) : (odd ? -pub : pwb);
    const float sp = p >= 0.f ? 1.f : -1.f;
    if (!of_b) {
        gx = sp * ax;
        gy = sp * ay;
        gt = -rd - (on_a ? sp * dp : 0.f);
    } else {
        gx = -sp * ax;
        gy = -sp * ay;
        gt = rd - (on_a ? 0.f : sp * dp);
    }
    return m;
}

// Corner k of a box: 0 front-left, 1 front-right, 2 rear-right, 3 rear-left.
__device__ __forceinline__ void box_corner(float x, float y, float c, float s, float hl, float hw, int k,
                                           float &cx, float &cy)
{
    const float sl = (k < 2) ? hl : -hl;
    const float sw = (k == 0 || k == 3) ? hw : -hw;
    cx = x + __builtin_fmaf(sl, c, -(sw * s));
    cy = y + __builtin_fmaf(sl, s, sw * c);
}

// Squared distance used by the off-road scan and its rescan (identical code
// in both places, so equal inputs give equal bits).
__device__ __forceinline__ float edge_d2(float qx, float qy, float cx, float cy)
{
    const float dx = qx - cx, dy = qy - cy;
    return __builtin_fmaf(dy, dy, dx * dx);
}

// ---------------------------------------------------------------------------
// Off-road scan (the hot loop).  A wave scans chunks [c0, c1) of one
// scenario's compacted road-edge stream (Edges) against R corners held per
// lane.  Each chunk passes once through the wave's LDS stage and reaches all
// 64 lanes as broadcast reads.
//
// The inner loop evaluates the expanded form
//     T(q) = |q|^2 - 2 c.q  ( = |q - c|^2 - |c|^2 )
// as fma(-2cy, qy, fma(-2cx, qx, qq)): two FMAs and half a v_min3 per
// (corner, point).  T is only used to select candidate chunks: per corner the
// three smallest chunk minima are kept (values b1 <= b2 <= b3, chunk indices
// of the first two).  Rounding of T and of the direct distance
// D = fl(fl(dx^2) + dy^2) are both below 4u (|q| + |c|)^2 (u = 2^-24), so any
// chunk whose T-minimum exceeds the best one by more than
//     delta = 2^-19 (Rq + |c|)^2      (Rq = max |q| of the scenario)
// cannot hold a point whose D is the minimum.  The candidate chunks (one or
// two; with three or more, every point) are then rescanned with D, and the
// lowest index of the minimum of D is the nearest point -- the same result as
// an exact scan of D over all points.
// ---------------------------------------------------------------------------
constexpr int kChunkFloats = 3 * kChunk;

__device__ __forceinline__ float candidate_band(float qqmax, float cx, float cy)
{
    const float r = sqrtf(qqmax) + sqrtf(__builtin_fmaf(cy, cy, cx * cx));
    return 0x1p-19f * r * r;
}

// Bytes of the per-wave LDS stage of the scan (one chunk).
constexpr int kStageBytes = kChunkFloats * 4;

// Position of point j's qq in its chunk's qq column: rotated by one within
// each group of four.  A 16-byte LDS read puts component c of a group in a
// register of VGPR bank c, so point j's x (component j % 4) and its qq
// (component (j + 1) % 4) come from different banks and the FMA that reads
// both does not stall on a bank conflict.
__host__ __device__ constexpr int qq_slot(int j) { return (j & ~3) | ((j + 1) & 3); }

// Minimum of T over one chunk already staged in LDS (x, y, qq columns),
// folded into m.  All lanes read the same addresses (LDS broadcast reads of
// four points per column); the points are VGPR operands of the FMAs.
template <int R>
__device__ __forceinline__ void fold_chunk(const float4 *stage, const float (&m2x)[R],
                                           const float (&m2y)[R], float (&m)[R])
{
#pragma unroll 4
    for (int j4 = 0; j4 < kChunk / 4; ++j4) {
        const float4 X = stage[j4], Y = stage[kChunk / 4 + j4], Q = stage[kChunk / 2 + j4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // Q holds the group's qq rotated by one (qq_slot)
            const float t0 = __builtin_fmaf(m2y[r], Y.x, __builtin_fmaf(m2x[r], X.x, Q.y));
            const float t1 = __builtin_fmaf(m2y[r], Y.y, __builtin_fmaf(m2x[r], X.y, Q.z));
            const float t2 = __builtin_fmaf(m2y[r], Y.z, __builtin_fmaf(m2x[r], X.z, Q.w));
            const float t3 = __builtin_fmaf(m2y[r], Y.w, __builtin_fmaf(m2x[r], X.w, Q.x));
            m[r] = fminf(fminf(m[r], t0), t1);
            m[r] = fminf(fminf(m[r], t2), t3);
        }
    }
}

// Scan of chunks [c0, c1) by one wave for R corner sets per lane.  The wave
// stages each chunk through its own LDS stage (`stage`, kStageBytes): every
// lane fetches its 16-byte pieces of the next chunk into registers while the
// current one is folded (global loads complete in order, so the fetch stays
// in flight), then writes them to the stage once the current chunk has been
// read, and all lanes read the chunk back as broadcasts.  A wave's LDS
// operations execute in order, so one stage suffices.  Keeps per corner the
// three smallest chunk minima and the chunks of the first two.
template <int R>
__device__ __forceinline__ void scan_edges(const float *__restrict__ stream, int c0, int c1, float4 *stage,
                                           const float (&cx)[R], const float (&cy)[R], float (&b1)[R],
                                           float (&b2)[R], float (&b3)[R], int (&i1)[R], int (&i2)[R])
{
    if (c0 >= c1)
        return;
    constexpr int kC4 = kStageBytes / 16;             // float4 per chunk
    static_assert(kC4 > 64 && kC4 <= 128, "two 16-byte pieces per lane");
    const int lane = threadIdx.x & 63;
    const bool second = lane < kC4 - 64;
    const float4 *src = (const float4 *)stream + lane;
    float m2x[R], m2y[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        m2x[r] = -2.0f * cx[r];
        m2y[r] = -2.0f * cy[r];
    }
    float4 va = src[(long)kC4 * c0], vb = make_float4(0.f, 0.f, 0.f, 0.f);
    if (second)
        vb = src[(long)kC4 * c0 + 64];
    for (int c = c0; c < c1; ++c) {
        stage[lane] = va;
        if (second)
            stage[64 + lane] = vb;
        if (c + 1 < c1) {
            va = src[(long)kC4 * (c + 1)];
            if (second)
                vb = src[(long)kC4 * (c + 1) + 64];
        }
        float m[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            m[r] = __builtin_inff();
        fold_chunk<R>(stage, m2x, m2y, m);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // selects on the two comparisons keep the update branch-free
            const bool lt1 = m[r] < b1[r], lt2 = m[r] < b2[r];
            b3[r] = __builtin_amdgcn_fmed3f(b2[r], b3[r], m[r]);
            b2[r] = __builtin_amdgcn_fmed3f(b1[r], b2[r], m[r]);
            b1[r] = lt1 ? m[r] : b1[r];
            const int j2 = lt2 ? c : i2[r];
            i2[r] = lt1 ? i1[r] : j2;
            i1[r] = lt1 ? c : i1[r];
        }
    }
}

// Lower bound of D = fl(fl(dx^2) + dy^2) (edge_d2) over the points of a box
// (xmin, xmax, ymin, ymax) for the corner (cx, cy): the box's nearest point,
// with the same roundings.  Rounding is monotone, so for every point q of
// the box |fl(qx - cx)| >= the bound's dx (likewise y) and D(q) >= the
// bound, bit for bit.  An empty box (+inf, -inf, ...) gives +inf.
__device__ __forceinline__ float box_lb(const float4 bb, float cx, float cy)
{
    const float lx = bb.x - cx, hx = bb.y - cx, ly = bb.z - cy, hy = bb.w - cy;
    // lx > 0 and hx < 0 exclude each other (xmin <= xmax; an empty box has
    // lx = +inf), so the larger of lx, -hx and 0 is the distance along x
    const float dx = fmaxf(fmaxf(lx, -hx), 0.f);
    const float dy = fmaxf(fmaxf(ly, -hy), 0.f);
    return __builtin_fmaf(dy, dy, dx * dx);
}

// The pruned scan (scan_group_pruned) stages up to kPruneBatch blocks at a
// time per wave; a staged block is its 32 points' x, y and qq, 8 float4 each
// (kBlockF4), and one more float4 takes the writes of the lanes that load
// nothing.  Per wave it also lists the needed blocks (kPruneList 16-bit
// entries).
constexpr int kPruneBatch = 8;
constexpr int kBlockF4 = 24;
constexpr int kPruneStageBytes = (kPruneBatch * kBlockF4 + 1) * 16;
constexpr int kPruneList = 512;
constexpr int kPruneWaveBytes = kPruneStageBytes + kPruneList * 2;

// Minimum over the lanes of a group of CL consecutive lanes (CL = 4, 8 or
// 16), in every lane of the group (quad swaps, then half-row and row
// mirrors).
template <int Ctrl>
__device__ __forceinline__ float dpp_min(float v)
{
    // every lane's source lane exists in these patterns, so bound_ctrl
    // changes nothing but spares the move of a default value; the median
    // with -FLT_MAX is the minimum of two values above it in one
    // instruction (fminf would first quiet the moved value, which is never
    // a NaN here)
    return __builtin_amdgcn_fmed3f(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), Ctrl, 0xF, 0xF, true)),
                                   -0x1.fffffep127f);
}

template <int CL>
__device__ __forceinline__ float lanes_min(float v)
{
    static_assert(CL == 4 || CL == 8 || CL == 16, "lane groups of 4, 8 or 16");
    v = dpp_min<0xB1>(v);       // quad_perm [1, 0, 3, 2]
    v = dpp_min<0x4E>(v);       // quad_perm [2, 3, 0, 1]
    if constexpr (CL >= 8)
        v = dpp_min<0x141>(v);  // row_half_mirror
    if constexpr (CL >= 16)
        v = dpp_min<0x140>(v);  // row_mirror
    return v;
}

// Maximum over the 16 lanes of a DPP row, in every lane of it.
template <int Ctrl>
__device__ __forceinline__ float dpp_max(float v)
{
    return fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), Ctrl, 0xF, 0xF, true)));
}

__device__ __forceinline__ float lanes_max16(float v)
{
    v = dpp_max<0xB1>(v);
    v = dpp_max<0x4E>(v);
    v = dpp_max<0x141>(v);
    return dpp_max<0x140>(v);
}

// Sum over the lanes of a group of 8 consecutive lanes, in every lane of it.
template <int Ctrl>
__device__ __forceinline__ int dpp_add(int v)
{
    return v + __builtin_amdgcn_mov_dpp(v, Ctrl, 0xF, 0xF, true);
}

__device__ __forceinline__ int lanes_sum8(int v)
{
    v = dpp_add<0xB1>(v);
    v = dpp_add<0x4E>(v);
    return dpp_add<0x141>(v);
}

// Minimum of T over this lane's PL points (part `part`) of a staged block,
// folded into m.
template <int PL>
__device__ __forceinline__ void fold_part(const float4 *st, int part, float m2x, float m2y, float &m)
{
#pragma unroll
    for (int q = 0; q < PL / 4; ++q) {
        const int j4 = part * (PL / 4) + q;
        const float4 X = st[j4], Y = st[8 + j4], Q = st[16 + j4];
        // Q holds the group's qq rotated by one (qq_slot)
        const float t0 = __builtin_fmaf(m2y, Y.x, __builtin_fmaf(m2x, X.x, Q.y));
        const float t1 = __builtin_fmaf(m2y, Y.y, __builtin_fmaf(m2x, X.y, Q.z));
        const float t2 = __builtin_fmaf(m2y, Y.z, __builtin_fmaf(m2x, X.z, Q.w));
        const float t3 = __builtin_fmaf(m2y, Y.w, __builtin_fmaf(m2x, X.w, Q.x));
        m = fminf(fminf(m, t0), t1);
        m = fminf(fminf(m, t2), t3);
    }
}

// The block minima of the road-edge scan for the 4 GO corners of a group of
// GO objects, with whole blocks of 32 points skipped.  Corner k is held by
// the CL = 16 / GO lanes k CL .. k CL + CL - 1 (each with the corner's cx,
// cy and thr); a lane folds PL = 32 / CL points of each block, and the
// lanes' minima are combined per block.  On return every lane of a corner
// holds its (b1, b2, b3, i1, i2): the three smallest block minima of T over
// the folded blocks and the blocks (index 4 chunk + block) of the first two,
// as scan_edges keeps them per chunk.
//
// thr bounds what the corner still needs: a block whose box_lb exceeds thr
// for every corner of the group is neither loaded nor folded.  The caller
// sets thr = D(corner, q) + 2 band for a point q it knows (or +inf): the
// block of q is then always folded, so the chunk minima kept here include
// the overall minimum of T, and every skipped point has T above that minimum
// plus the band (T and D agree within a quarter band), so no chunk with
// skipped points only could have been a candidate.  -inf marks a corner that
// needs nothing.
//
// The tests run with a box per lane: per pass of 64 chunks, lane j tests
// chunk box j against every object of the group (broadcast from its lanes):
// its centre (ox, oy) and the radius orad of the circle through its corners
// give a bound that every corner's test implies (below); then lane l tests
// block l & 3 of the (l >> 2)-th chunk that passed, 16 such chunks at a
// time, against every corner; the needed blocks are listed in ascending
// order and fetched
// kPruneBatch at a time, two per 16-byte load (lanes 0..47), the next batch
// in flight while one is folded from `stage`.  cbox and box may point to
// global memory or to a copy in LDS.
// Work counts of the pruned scan (wave-uniform): blocks folded, chunk boxes
// tested against an object, block boxes tested against a corner.
struct ScanCounts {
    uint32_t folded, chunk_tests, block_tests;
};

template <int GO>
__device__ __forceinline__ void scan_group_pruned(const float *__restrict__ stream, const float4 *cbox,
                                                  const float4 *box, int nch, float4 *stage, uint16_t *list,
                                                  float cx, float cy, float thr, float ox, float oy, float orad,
                                                  float &b1, float &b2, float &b3, int &i1, int &i2,
                                                  ScanCounts &work)
{
    constexpr int NC = 4 * GO, CL = 64 / NC, PL = 32 / CL;
    static_assert(NC * CL == 64 && 4 * CL == 16, "an object's corners fill one DPP row of 16 lanes");
    constexpr int kChunkF4 = kStageBytes / 16;   // float4 per chunk in the stream
    static_assert(kChunk == 4 * 32 && kChunkF4 == 3 * 32, "four blocks of 32 points per chunk");
    static_assert(PL % 4 == 0, "whole groups of four points per lane");
    static_assert(kPruneBatch % 2 == 0 && 2 * kBlockF4 <= 64, "two blocks per load");
    const int lane = threadIdx.x & 63, part = lane % CL;
    const float4 *src = (const float4 *)stream;
    const float4 empty = make_float4(__builtin_inff(), -__builtin_inff(), __builtin_inff(), -__builtin_inff());
    const float m2x = -2.0f * cx, m2y = -2.0f * cy;
    // is this lane's box needed by some corner of the group
    auto any_corner = [&](const float4 b) -> bool {
        bool a = false;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const float kx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cx), k * CL));
            const float ky = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cy), k * CL));
            const float kt = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(thr), k * CL));
            a |= box_lb(b, kx, ky) <= kt;
        }
        return a;
    };
    // The object bound.  A corner c passes box B when box_lb(B, c) <= thr_c;
    // then the exact distance d(B, c) <= sqrt(thr_c) (1 + 2 eps) (box_lb
    // rounds its three operations down by at most a factor (1 - eps)^3), so
    // d(B, centre) <= d(B, c) + |c - centre| <= sqrt(thr_max) (1 + 2 eps) +
    // orad + (rounding of the corner), and box_lb(B, centre) is at most
    // (1 + eps)^3 times its square.  The relative 2^-10 and the absolute
    // 1e-3 m + 2^-20 (|ox| + |oy|) margins cover all of these, and a chunk
    // box contains its blocks' boxes, so a chunk failing the bound has no
    // block any corner needs.
    const float tmax = lanes_max16(thr);
    float othr = -__builtin_inff();
    if (tmax >= 0.f) {
        const float rr = sqrtf(tmax) * (1.0f + 0x1p-10f) + orad + 1e-3f + 0x1p-20f * (fabsf(ox) + fabsf(oy));
        othr = rr * rr;
    }
    auto any_object = [&](const float4 b) -> bool {
        bool a = false;
#pragma unroll
        for (int j = 0; j < GO; ++j) {
            const float kx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ox), 16 * j));
            const float ky = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(oy), 16 * j));
            const float kt = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(othr), 16 * j));
            a |= box_lb(b, kx, ky) <= kt;
        }
        return a;
    };

    // block cur's minimum mm (over all its lanes) into the three smallest
    auto push = [&](float mm, int cur) {
        const bool lt1 = mm < b1, lt2 = mm < b2;
        b3 = __builtin_amdgcn_fmed3f(b2, b3, mm);
        b2 = __builtin_amdgcn_fmed3f(b1, b2, mm);
        b1 = lt1 ? mm : b1;
        const int j2 = lt2 ? cur : i2;
        i2 = lt1 ? i1 : j2;
        i1 = lt1 ? cur : i1;
    };
    // this lane's piece of a block: column (x, y, qq) piece / 8, float4 piece % 8
    const int half = lane / kBlockF4, piece = lane % kBlockF4;
    const int poff = (piece / 8) * (kChunk / 4) + piece % 8;
    const bool loader = half < 2;
    int seg = 0;    // list entries are 4 (chunk - seg) + block
    int nl = 0;
    // the batch in flight: slot s holds blocks 2 s (lanes 0..23) and 2 s + 1
    // (lanes 24..47) of the batch (four named slots, so that they stay in
    // registers)
    static_assert(kPruneBatch == 8, "four load slots");
    float4 v0, v1, v2, v3;
    // every lane loads (those without a block of their own the batch's
    // first one again), so that no lane-dependent branch leaves a load
    // pending
    auto load_slot = [&](int b0, int nb, int s) -> float4 {
        const int i = 2 * s + half;
        const int e = list[b0 + (loader && i < nb ? i : 0)];
        return src[(long)kChunkF4 * (seg + (e >> 2)) + (e & 3) * 8 + poff];
    };
    auto fetch = [&](int b0, int nb) {
        v0 = load_slot(b0, nb, 0);
        if (nb > 2)
            v1 = load_slot(b0, nb, 1);
        if (nb > 4)
            v2 = load_slot(b0, nb, 2);
        if (nb > 6)
            v3 = load_slot(b0, nb, 3);
    };
    const int sl = loader ? lane : kPruneBatch * kBlockF4;   // this lane's stage slot (or the spare float4)
    auto fold_list = [&]() {
        __builtin_amdgcn_wave_barrier();
        if (nl == 0)
            return;
        work.folded += nl;
        fetch(0, min(kPruneBatch, nl));
        for (int b0 = 0; b0 < nl; b0 += kPruneBatch) {
            const int nb = min(kPruneBatch, nl - b0);
            stage[sl] = v0;
            if (nb > 2)
                stage[loader ? 2 * kBlockF4 + sl : sl] = v1;
            if (nb > 4)
                stage[loader ? 4 * kBlockF4 + sl : sl] = v2;
            if (nb > 6)
                stage[loader ? 6 * kBlockF4 + sl : sl] = v3;
            if (b0 + kPruneBatch < nl)
                fetch(b0 + kPruneBatch, min(kPruneBatch, nl - b0 - kPruneBatch));
            __builtin_amdgcn_wave_barrier();
            const int ent = lane < nb ? (int)list[b0 + lane] : 0;   // the batch's entries, one per lane
            // two blocks at a time (for an odd count the second is a stale stage
            // slot, folded but not pushed)
            for (int i = 0; i < nb; i += 2) {
                float ma = __builtin_inff(), mb = __builtin_inff();
                fold_part<PL>(stage + kBlockF4 * i, part, m2x, m2y, ma);
                fold_part<PL>(stage + kBlockF4 * (i + 1), part, m2x, m2y, mb);
                ma = lanes_min<CL>(ma);
                mb = lanes_min<CL>(mb);
                push(ma, 4 * seg + __builtin_amdgcn_readlane(ent, i));
                if (i + 1 < nb)
                    push(mb, 4 * seg + __builtin_amdgcn_readlane(ent, i + 1));
            }
            __builtin_amdgcn_wave_barrier();
        }
        nl = 0;
    };
    for (int base = 0; base < nch; base += 64) {
        // room for a whole pass (256 entries) within 16-bit entries
        if (nl > kPruneList - 256 || base + 64 - seg > 16384)
            fold_list();
        if (nl == 0)
            seg = base;
        const int cnt = min(64, nch - base);
        const float4 cb = lane < cnt ? cbox[base + lane] : empty;
        // bit j: chunk base + j may hold a needed point (lanes past the range
        // hold an empty box, which a corner with thr = +inf would pass)
        uint64_t cm = __ballot(lane < cnt && any_object(cb));
        work.chunk_tests += GO * cnt;
        while (cm != 0) {
            // lane l: block (l & 3) of the (l >> 2)-th needed chunk of this batch
            int myc = -1;
            int nb = 0;
            for (; nb < 16 && cm != 0; ++nb) {
                const int j = __builtin_ctzll(cm);
                cm &= cm - 1;
                if ((lane >> 2) == nb)
                    myc = base + j;
            }
            work.block_tests += NC * 4 * nb;
            const float4 bb = myc >= 0 ? box[4 * myc + (lane & 3)] : empty;
            const uint64_t bm = __ballot(myc >= 0 && any_corner(bb));   // bit l: lane l's block is needed
            const int below =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0));
            if ((bm >> lane) & 1ull)
                list[nl + below] = (uint16_t)(4 * (myc - seg) + (lane & 3));
            nl += __popcll(bm);
        }
    }
    fold_list();
}

// Exact rescan of part rl (of kBlockRescanLanes) of block `blk` (points
// 32 blk ..) for one corner, as rescan_part does for a chunk: the lowest
// index of the minimum of D over the part's real points (index < E), folded
// into (best, bidx) with strict <, the points in ascending order.
constexpr int kBlockRescanLanes = 4;
constexpr int kBlockRescanPart = 32 / kBlockRescanLanes;   // 8 points

__device__ __forceinline__ void rescan_block(const float *__restrict__ stream, int blk, int rl, int E, float cx,
                                             float cy, float &best, int &bidx)
{
    const int j0 = 32 * blk + rl * kBlockRescanPart;   // first point of the part
    const float *col = stream + kChunkFloats * (blk >> 2) + 32 * (blk & 3) + rl * kBlockRescanPart;
    const float4 *px = (const float4 *)col, *py = (const float4 *)(col + kChunk);
    const int n = E - j0;   // points of this part inside the stream
#pragma unroll
    for (int b = 0; b < kBlockRescanPart / 4; ++b) {
        const float4 X = px[b], Y = py[b];
        const float xs[4] = {X.x, X.y, X.z, X.w}, ys[4] = {Y.x, Y.y, Y.z, Y.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int j = 4 * b + k;
            const float d = edge_d2(xs[k], ys[k], cx, cy);
            if (j < n && d < best) {
                best = d;
                bidx = j0 + j;
            }
        }
    }
}

// Exact rescan of part rl (of kRescanLanes) of chunk `c` for one corner:
// the lowest index of the minimum of D over the part's real points (index <
// E), points c * kChunk + rl * kRescanPart + k in ascending k, folded into
// (best, bidx) with strict <; a (D, index) reduction over the parts then
// gives the chunk's lowest-index minimum, and chunks rescanned in ascending
// order keep the lowest index.  The x and y columns arrive as 16-byte vector
// loads (chunks are 16-byte aligned in the workspace).
constexpr int kRescanLanes = 8;
constexpr int kRescanPart = kChunk / kRescanLanes;   // 16 points
static_assert(kRescanPart % 4 == 0, "a part is whole float4 groups");

__device__ __forceinline__ void rescan_part(const float *__restrict__ stream, int c, int rl, int E, float cx,
                                            float cy, float &best, int &bidx)
{
    const float4 *px = (const float4 *)(stream + kChunkFloats * c) + rl * (kRescanPart / 4);
    const float4 *py = (const float4 *)(stream + kChunkFloats * c + kChunk) + rl * (kRescanPart / 4);
    const int n = E - kChunk * c - rl * kRescanPart;   // points of this part inside the stream
#pragma unroll
    for (int b = 0; b < kRescanPart / 4; ++b) {
        const float4 X = px[b], Y = py[b];
        const float xs[4] = {X.x, X.y, X.z, X.w}, ys[4] = {Y.x, Y.y, Y.z, Y.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int j = 4 * b + k;
            const float d = edge_d2(xs[k], ys[k], cx, cy);
            if (j < n && d < best) {
                best = d;
                bidx = kChunk * c + rl * kRescanPart + j;
            }
        }
    }
}

} // namespace wm
