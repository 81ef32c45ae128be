/*
 * wm.h -- C ABI of the MI355X (gfx950) simulator hot path.
 *
 * The library implements the batched simulator step of "Waymax: An
 * Accelerated, Data-Driven Simulator for Large-Scale Autonomous Driving
 * Research" (arXiv 2310.08710) with hand-written HIP kernels:
 *   - kinematic bicycle dynamics, forward and inverse, and the delta action
 *     space (App. A.1); discretized actions (Sec. 5.2),
 *   - the per-step metrics of Sec. 3.4: collision (box overlap), off-road
 *     (side of the nearest oriented road edge), displacement error and
 *     kinematic infeasibility, plus the sparse reward of Sec. 5.2,
 *   - the default observation of Sec. 3.2 (ego frame + k nearest road points),
 *     for one state or every step of a state sequence,
 *   - fused multi-step rollouts (Sec. 5.1, Rollout), with log playback or IDM
 *     sim agents (Sec. 3.5), and their adjoint (differentiable simulation,
 *     Sec. 1 and Sec. 6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array pointers are DEVICE pointers owned by the caller.  The library
 *    never allocates, frees or retains caller memory; scratch memory comes
 *    from the caller-provided workspace (see wm_workspace_bytes).
 *  - Every call validates its host-visible arguments synchronously, BEFORE
 *    any launch, and returns a WM_ERR_* code without touching the device on
 *    failure.  Device array contents (offsets, flags) are trusted.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    the call returns without synchronizing.  Calls contain no host-device
 *    synchronization, no allocation and no memset, so a sequence of them can
 *    be captured into a HIP graph (wm_autotune, which times launches, is the
 *    exception).
 *  - Batches are packed (CSR): scenario s owns objects obj_off[s] ..
 *    obj_off[s+1]-1 and road points rg_off[s] .. rg_off[s+1]-1 of the global
 *    arrays.  Objects of different scenarios never interact.
 *  - States are structure-of-arrays float32 + a uint8 valid flag.  A state
 *    sequence (logs, trajectories, checkpoints) is time-major: field[t * n + i]
 *    with n = wm_batch.total_objects.
 *  - Units: metres, radians, seconds.  Length is measured along the yaw; boxes
 *    are centred on (x, y).
 *  - A metric triggers iff its margin is strictly positive.  Margins with no
 *    defined value (invalid object, no partner, no road edge) are -FLT_MAX.
 *  - Road-point indices (nearest_idx, rg_idx) are scenario-local.
 *  - Errors: the return value is WM_OK or a WM_ERR_* code; a thread-local
 *    message with the detail is available from wm_last_error_message().
 */
#ifndef WM_H
#define WM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define WM_OK 0
#define WM_ERR_NULL 1        /* a required pointer is NULL */
#define WM_ERR_RANGE 2       /* a scalar is out of range (S, T, k, E < 1; dt <= 0 or not finite ...) */
#define WM_ERR_SHAPE 3       /* inconsistent sizes (totals, maxima) */
#define WM_ERR_WORKSPACE 4   /* workspace missing or smaller than wm_workspace_bytes */
#define WM_ERR_UNSUPPORTED 5 /* a size beyond what the kernels support (see limits) */
#define WM_ERR_DEVICE 6      /* a HIP runtime error; the message carries hipGetErrorString */

/* Limits. */
#define WM_MAX_OBJECTS 1024      /* objects per scenario */
#define WM_MAX_TOPK 1024         /* k of wm_observe */
#define WM_MAX_OBSERVE_POINTS 32768 /* road points per scenario for wm_observe */
#define WM_MAX_IDM_POSES 64      /* lookahead poses of wm_rollout_idm */

/* Road-point type of an oriented road edge (Sec. 3.4, Off-Road). */
#define WM_TYPE_ROAD_EDGE 1

/* A packed batch of scenarios.  The int32 fields are host values; obj_off and
 * rg_off are device arrays of S+1 non-decreasing entries starting at 0.
 * max_objects / max_rg_points must be >= every scenario's count (they size
 * launches and shared memory); total_objects = obj_off[S] and
 * total_rg_points = rg_off[S]. */
typedef struct wm_batch {
    int32_t num_scenarios;
    int32_t total_objects;
    int32_t total_rg_points;
    int32_t max_objects;
    int32_t max_rg_points;
    const int32_t *obj_off;
    const int32_t *rg_off;
} wm_batch;

/* Dynamic object state (Sec. 3.2: position, rotation, velocity, box
 * dimensions; plus validity).  Each member points to total_objects entries
 * (or T * total_objects for a sequence). */
typedef struct wm_state {
    float *x, *y, *yaw, *vx, *vy, *length, *width;
    uint8_t *valid;
} wm_state;

/* Static road graph (Sec. 3.2; oriented points, Sec. 3.4 Off-Road), one
 * entry per point: position, unit direction, type (WM_TYPE_ROAD_EDGE for
 * road edges), validity.  2D: elevation is not used by any metric. */
typedef struct wm_roadgraph {
    const float *x, *y, *dir_x, *dir_y;
    const int8_t *type;
    const uint8_t *valid;
} wm_roadgraph;

/* Bicycle actions (App. A.1: acceleration a [m/s^2], curvature kappa [1/m])
 * plus the control mask of Sec. 4.1 / Sec. 4.3: objects with controlled = 0
 * replay the log instead.  accel/curvature hold total_objects entries for a
 * step, T * total_objects (time-major) for a rollout; controlled always holds
 * total_objects entries (constant over a rollout). */
typedef struct wm_action {
    const float *accel, *curvature;
    const uint8_t *controlled;
} wm_action;

/* Per-object metrics of one step (Sec. 3.4); T * total_objects entries for a
 * rollout.  Any member may be NULL (not computed / not written).
 *   collision       1 iff the box overlaps another valid box of the scenario
 *   overlap_margin  max over partners of the separating-axis margin
 *   offroad         1 iff some box corner lies right of its nearest road edge
 *   offroad_margin  max over the 4 corners of the signed side distance
 *   log_div         |xy - xy_log| when both are valid, else 0
 *   infeasible      kinematic infeasibility of the transition into this state
 *                   (Sec. 3.4): the bicycle inverse of (previous, successor)
 *                   has |a| > 6 m/s^2 or |kappa| > 0.3 1/m; 0 unless both
 *                   states are valid
 *   reward          -1[collision] - 1[off-road] (the sparse reward of Sec. 5.2);
 *                   requires collision and, with a road graph, offroad */
typedef struct wm_metrics {
    uint8_t *collision, *offroad;
    float *overlap_margin, *offroad_margin, *log_div;
    uint8_t *infeasible;
    float *reward;
} wm_metrics;

/* Optional launch tuning of the off-road / rollout kernels; NULL selects the
 * library's choice (autotuned table if wm_autotune has run, else a default).
 *   unit_objects  objects per work unit (one work-group): 64, 128 or 256
 *   edge_splits   1, 2, 4, 8 or 16: the work-group's waves per 64
 *                 objects.  In the rollouts, and in wm_offroad / wm_step
 *                 with a work-group of at most 512 threads, they claim the
 *                 unit's groups of four objects for the pruned off-road
 *                 scan; in wm_offroad with a larger work-group (the scan of
 *                 every point), they scan that many road-edge ranges of
 *                 each object in parallel
 * unit_objects * edge_splits (the work-group size) must not exceed 1024 for
 * wm_offroad and 512 for wm_rollout / wm_autotune; larger values fail with
 * WM_ERR_RANGE. */
typedef struct wm_tuning {
    int32_t unit_objects;
    int32_t edge_splits;
} wm_tuning;

/* Bytes of device workspace needed by any call on this batch.  T = 0 covers
 * the single-step calls; a rollout needs its own T and ckpt_every (0 = no
 * checkpoints).  Returns 0 if the batch is invalid. */
size_t wm_workspace_bytes(const wm_batch *batch, int32_t T, int32_t ckpt_every);

/* The same number under the name of the rollout's workspace query: bytes of
 * workspace for wm_rollout / wm_rollout_backward with this T and checkpoint
 * interval (every other call on the batch fits in it too). */
size_t wm_rollout_workspace_bytes(const wm_batch *batch, int32_t T, int32_t ckpt_every);

/* One simulator step (Sec. 4.1 step(state, action); dynamics App. A.1
 * bicycle forward).  For every object:
 *   controlled & valid   : bicycle forward with (accel, curvature)
 *   controlled & invalid : frozen (next = cur)
 *   not controlled       : next = log_next (log playback, Sec. 4.3)
 * Metrics, if m != NULL, are evaluated on the successor state `next`
 * (collision and off-road need the whole scenario; off-road is skipped when
 * rg == NULL).  `next` must not alias `cur`.  Workspace: wm_workspace_bytes(batch, 0, 0)
 * when off-road metrics are requested, else may be NULL. */
int wm_step(const wm_batch *batch, const wm_state *cur, const wm_action *act,
            const wm_state *log_next, const wm_roadgraph *rg, float dt, wm_state *next,
            wm_metrics *m, void *ws, size_t ws_bytes, void *stream);

/* Step-by-step simulation with a fixed road graph (closed-loop use, Sec. 4.1):
 * wm_roadgraph_prepare compacts the road edges of `rg` into `ws` once (the
 * first part of every off-road computation, which wm_step repeats at each
 * call); wm_step_prepared is wm_step without that compaction.  Precondition
 * of wm_step_prepared: the last compaction into `ws` (by
 * wm_roadgraph_prepare, wm_step, wm_offroad or wm_rollout) was of the same
 * batch and road graph, which have not changed since; otherwise its
 * off-road outputs are undefined (no fault: every index stays inside the
 * workspace).  Workspace: wm_workspace_bytes(batch, 0, 0). */
int wm_roadgraph_prepare(const wm_batch *batch, const wm_roadgraph *rg, void *ws, size_t ws_bytes, void *stream);
int wm_step_prepared(const wm_batch *batch, const wm_state *cur, const wm_action *act, const wm_state *log_next,
                     const wm_roadgraph *rg, float dt, wm_state *next, wm_metrics *metrics, void *ws,
                     size_t ws_bytes, void *stream);

/* Bytes of the device-resident workspace of wm_step_noalloc: one copy per
 * device the library runs on, held until the process ends. */
#define WM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* wm_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and outputs as wm_step, with the workspace taken from a device
 * array of WM_NOALLOC_SCRATCH_BYTES that the library holds instead of a ws
 * argument.  Calls no hipMalloc, hipFree or allocating library routine; the
 * first call on a device looks up that device's array address (a host-side
 * query, not a stream operation).  Fails with WM_ERR_UNSUPPORTED, before any
 * launch, when off-road metrics are requested and wm_workspace_bytes(batch,
 * 0, 0) exceeds WM_NOALLOC_SCRATCH_BYTES (64 MiB holds about 2.7 million road
 * points per batch).  Every call on one device shares that device's array and
 * it keeps the last call's contents (nothing in it needs to start at zero):
 * calls that overlap in time on one device (several streams or threads) race
 * on it, so the caller must order them, e.g. on one stream. */
int wm_step_noalloc(const wm_batch *batch, const wm_state *cur, const wm_action *act, const wm_state *log_next,
                    const wm_roadgraph *rg, float dt, wm_state *next, wm_metrics *metrics, void *stream);

/* Expert action by inverse kinematics (App. A.1, inverse kinematics
 * equation; Sec. 5.2 Expert): a = (|v'| - |v|)/dt,
 * kappa = wrap(atan2(vy', vx') - yaw) / (|v| dt + a dt^2/2), kappa = 0 when
 * that distance is below 1e-6 m.  valid_out = both states valid (a = kappa = 0
 * otherwise).  Outputs hold total_objects entries; valid_out may be NULL. */
int wm_inverse_action(const wm_batch *batch, const wm_state *cur, const wm_state *next, float dt,
                      float *accel, float *curvature, uint8_t *valid_out, void *stream);

/* Delta actions (App. A.1, delta action space): increments of x, y and yaw
 * per step ([total_objects] each) plus the control mask, as for wm_action. */
typedef struct wm_delta_action {
    const float *dx, *dy, *dyaw;
    const uint8_t *controlled;
} wm_delta_action;

/* One step in the delta action space (App. A.1, delta equations):
 * x' = x + dx, y' = y + dy, yaw' = yaw + dyaw, (vx', vy') = ((x' - x), (y' - y)) / dt,
 * with the control semantics of wm_step (playback / frozen).  Dynamics only:
 * metrics of `next` come from wm_overlap / wm_offroad. */
int wm_step_delta(const wm_batch *batch, const wm_state *cur, const wm_delta_action *act,
                  const wm_state *log_next, float dt, wm_state *next, void *stream);

/* Inverse of the delta step (App. A.1): (dx, dy, dyaw) = s' - s; zero and
 * valid_out = 0 unless both states are valid.  valid_out may be NULL. */
int wm_inverse_delta(const wm_batch *batch, const wm_state *cur, const wm_state *next, float *dx, float *dy,
                     float *dyaw, uint8_t *valid_out, void *stream);

/* Discretized actions (Sec. 5.2, Expert: the discrete inverse is the
 * continuous inverse discretized): each of the n values maps to the nearest
 * of `bins` (>= 2) evenly spaced values over [lo, hi] (lo < hi, finite);
 * half-way values go to the upper one, values outside the range to the end
 * bins.  Decided in binary32 as index = floor((v - lo) * s + 0.5) with
 * s = fl((bins - 1) / (hi - lo)); snapped = lo + index * fl((hi - lo) / (bins - 1)).
 * values/index/snapped are device arrays of n entries; snapped may be NULL. */
int wm_discretize(const float *values, int32_t n, float lo, float hi, int32_t bins, int32_t *index,
                  float *snapped, void *stream);

/* Collision metric (Sec. 3.4, Collision: 2D top-down box overlap) by the
 * separating-axis test.  For every object: collision (u8) and max_margin
 * (f32), either may be NULL.  Optionally the full per-scenario margin / mask
 * matrices: block s starts at pair_off[s] (device int64 [S+1]) and holds
 * N_s x N_s row-major entries (diagonal and pairs with an invalid box:
 * margin -FLT_MAX, mask 0).  margin and mask may be NULL; pair_off is required
 * iff one of them is given.  The matrix is exactly symmetric. */
int wm_overlap(const wm_batch *batch, const wm_state *st, const int64_t *pair_off, float *margin,
               uint8_t *mask, uint8_t *collision, float *max_margin, void *stream);

/* Off-road metric (Sec. 3.4, Off-Road).  For each of the 4 corners of every
 * valid box (front-left, front-right, rear-right, rear-left) the nearest valid
 * road-edge point q (2D distance, ties to the lower index) decides the side:
 * s = -cross(dir_q, corner - q) > 0 means off road.  margin = max_k s_k,
 * offroad = margin > 0.  nearest_idx (int32 [4 * total_objects], may be NULL)
 * receives the scenario-local index per corner (-1: none).  Workspace:
 * wm_workspace_bytes(batch, 0, 0).  `tune` may be NULL. */
int wm_offroad(const wm_batch *batch, const wm_state *st, const wm_roadgraph *rg, uint8_t *offroad,
               float *margin, int32_t *nearest_idx, const wm_tuning *tune, void *ws, size_t ws_bytes,
               void *stream);

/* Default observation (Sec. 3.2): for each of the E egos of every scenario
 * (ego: device int32 [S * E], global object ids):
 *   rg_idx   int32 [S*E*k]: the k valid road points (any type) nearest to the
 *            ego centre, ascending by (d2, index) with the binary32 key
 *            d2 = fl(fl(dx*dx) + fl(dy*dy)), dx = fl(qx - ex); -1 padding.
 *   rg_feat  f32 [S*E*k*4] or NULL: R(-yaw_e)(q - p_e), R(-yaw_e) dir_q; 0 padding.
 *   obj_feat f32 [S*E*max_objects*8] or NULL: for object j of the scenario,
 *            R(-yaw_e)(p_j - p_e), wrap(yaw_j - yaw_e), R(-yaw_e) v_j, length,
 *            width, 1; zeros for invalid or padded slots.
 * An invalid ego yields -1 / zeros.  Limits: k <= WM_MAX_TOPK,
 * max_rg_points <= WM_MAX_OBSERVE_POINTS. */
int wm_observe(const wm_batch *batch, const wm_state *st, const wm_roadgraph *rg, const int32_t *ego,
               int32_t E, int32_t k, int32_t *rg_idx, float *rg_feat, float *obj_feat, void *stream);

/* The default observation of every step of a state sequence in one launch:
 * for the paper's per-step observation (Sec. 4.1, step returns the next
 * observation) of a rollout's trajectory.  st holds T rows [T][n] (row t at
 * st + t * total_objects, e.g. the traj of wm_rollout); the egos are the same
 * for every row; row t's outputs follow row t-1's: rg_idx [T][S*E*k],
 * rg_feat [T][S*E*k*4], obj_feat [T][S*E*max_objects*8], each as in
 * wm_observe.  T <= 65535.  wm_observe is the case T = 1. */
int wm_observe_seq(const wm_batch *batch, const wm_state *st, int32_t T, const wm_roadgraph *rg, const int32_t *ego,
                   int32_t E, int32_t k, int32_t *rg_idx, float *rg_feat, float *obj_feat, void *stream);

/* One closed-loop simulator step (Sec. 4.1: step returns the successor
 * state, its metrics and the next observation): wm_step_prepared followed by
 * wm_observe of the successor `next` (the default observation of Sec. 3.2 for
 * the E egos of every scenario), in one call, with no host synchronization,
 * so that a policy loop can capture it in a HIP graph.  Arguments and outputs
 * as in those two calls: rg is required (the observation reads it); off-road
 * metrics read the road edges that wm_roadgraph_prepare compacted into `ws`
 * (same precondition as wm_step_prepared).  Every host-visible argument of
 * both parts is validated before the first launch. */
int wm_step_observe(const wm_batch *batch, const wm_state *cur, const wm_action *act, const wm_state *log_next,
                    const wm_roadgraph *rg, float dt, wm_state *next, wm_metrics *metrics, const int32_t *ego,
                    int32_t E, int32_t k, int32_t *rg_idx, float *rg_feat, float *obj_feat, void *ws,
                    size_t ws_bytes, void *stream);

/* Fused rollout of T steps (Sec. 5.1 Rollout; each step as wm_step with all
 * metrics, evaluated on the successor state).  One persistent kernel runs all
 * T steps of every (scenario, object slice) work unit, taking units from a
 * device queue in descending cost order.
 *   init       state at the current time (row 0 of the logs)
 *   act_seq    actions [T][n]; controlled [n]
 *   log_seq    logged states [T+1][n], row 0 = the initial time
 *   rg         road graph (off-road metrics); may be NULL (no off-road); the
 *              off-road scan runs only if met_seq requests offroad,
 *              offroad_margin or reward
 *   ckpt       [ceil(T/ckpt_every)][n] states at t = 0, c, 2c, ... or NULL
 *   traj       [T][n] successor states or NULL
 *   met_seq    [T][n] metrics or NULL (members may be NULL)
 *   loss       [S] training loss or NULL: sum over t of
 *                sum_{controlled i, valid in sim and log} |p_i - p_i^log|^2
 *              + sum_{i<j valid, i or j controlled} sigmoid(margin_ij / 0.1 m)
 * Workspace: wm_workspace_bytes(batch, T, ckpt_every). */
int wm_rollout(const wm_batch *batch, const wm_state *init, const wm_action *act_seq,
               const wm_state *log_seq, const wm_roadgraph *rg, int32_t T, float dt, int32_t ckpt_every,
               wm_state *ckpt, wm_state *traj, wm_metrics *met_seq, float *loss, const wm_tuning *tune,
               void *ws, size_t ws_bytes, void *stream);

/* Work counts of the off-road scan of the last wm_rollout or wm_rollout_idm
 * run with workspace `ws` (same batch), for measurement: counts[0] road-edge
 * blocks of 32 points folded (each for the 16 corners of a group of four
 * objects, so 512 corner-point evaluations), counts[1] chunk bounding boxes
 * tested against an object's circle, counts[2] block bounding boxes tested
 * against a corner (Sec. 3.4 Off-Road; the pruning is this library's, the
 * metric is unchanged).  `counts` is host memory [3]; the call waits for
 * `stream` to finish.  Errors: NULL pointers, a workspace smaller than the
 * counters' offset. */
int wm_rollout_scan_counts(const wm_batch *batch, const void *ws, size_t ws_bytes, uint64_t *counts, void *stream);

/* IDM sim agents (Sec. 3.5, simulated agent behaviour; intelligent driver
 * model of Treiber, Hennecke and Helbing 2000).  Field units: m, s. */
typedef struct wm_idm {
    float desired_speed;   /* v0 */
    float min_gap;         /* s0 */
    float time_headway;    /* T_h */
    float max_accel;       /* a_max */
    float comfort_decel;   /* b */
    float exponent;        /* delta */
    float max_brake;       /* hardest deceleration (> 0); also the response to a zero gap */
    float lookahead_step;  /* spacing of the lookahead poses along the path (> 0) */
    int32_t lookahead_poses; /* 1..WM_MAX_IDM_POSES */
} wm_idm;

/* Fused rollout as wm_rollout (no checkpoints, no loss) in which every
 * uncontrolled object whose log is valid in all rows 0..T is an IDM agent;
 * other uncontrolled objects replay the log, controlled ones follow act_seq.
 * An agent follows the polyline of its logged positions (rows 0..T, arc
 * length from row 0) with progress sigma (0 at t = 0).  Each step, with all
 * objects at time t-1:
 *   lead: lookahead poses at sigma + m * step (m = 1..poses, up to the path
 *     end) carry the agent's box; the lead is the valid object whose box
 *     overlaps (separating-axis margin > 0) the pose with the smallest m, then
 *     the lowest index; gap = (m - 1) * step; v_lead = its velocity along the
 *     agent's yaw.
 *   a = a_max (1 - (v / v0)^delta - (s_star / gap)^2), s_star = s0 +
 *     max(0, v T_h + v (v - v_lead) / (2 sqrt(a_max b))), no interaction
 *     term without a lead, -max_brake at gap 0, clamped to
 *     [-max_brake, a_max].
 *   v' = v + a dt, sigma += v dt + a dt^2 / 2 (or v^2 / (2|a|) and v' = 0 when
 *     stopping within the step); an agent reaching the path end halts there
 *     (sigma = path length, v' = 0); the pose at
 *     sigma: position interpolated linearly between logged rows, yaw between
 *     their yaws along the shorter arc; velocity v' along that yaw; length,
 *     width and valid from log row t.
 * Metrics as wm_rollout.  Workspace: wm_workspace_bytes(batch, T, 0). */
int wm_rollout_idm(const wm_batch *batch, const wm_state *init, const wm_action *act_seq,
                   const wm_state *log_seq, const wm_roadgraph *rg, int32_t T, float dt, const wm_idm *idm,
                   wm_state *traj, wm_metrics *met_seq, const wm_tuning *tune, void *ws, size_t ws_bytes,
                   void *stream);

/* Adjoint of wm_rollout's loss with respect to the actions (differentiable
 * simulation, Sec. 1 / Sec. 6), by a hand-written reverse sweep that
 * recomputes each checkpoint segment.  dloss [S] scales each scenario's loss
 * gradient.  grad_accel / grad_curvature [T][n] are overwritten (zero for
 * uncontrolled or invalid objects).  ckpt must come from wm_rollout with the
 * same inputs and ckpt_every.  Non-smooth points: sgn(0) = +1, the lowest
 * separating axis wins a tie, d|v|/dv = 0 at v = 0.  Workspace:
 * wm_workspace_bytes(batch, T, ckpt_every). */
int wm_rollout_backward(const wm_batch *batch, const wm_state *init, const wm_action *act_seq,
                        const wm_state *log_seq, int32_t T, float dt, int32_t ckpt_every,
                        const wm_state *ckpt, const float *dloss, float *grad_accel, float *grad_curvature,
                        void *ws, size_t ws_bytes, void *stream);

/* Measure the rollout for each candidate tuning on this batch (real launches
 * on `stream`, synchronizing) and remember the fastest for batches with the
 * same (max_objects, max_rg_points) bucket (power-of-two buckets).  best
 * (host) receives it; may be NULL.  Not capturable.  With the environment
 * variable WM_TUNE_CACHE naming a file, the pick is appended to that file
 * (one text line per device kind and bucket) and a later process takes a
 * matching line instead of timing again, also for a NULL tuning argument of
 * the rollout calls. */
int wm_autotune(const wm_batch *batch, const wm_state *init, const wm_action *act_seq,
                const wm_state *log_seq, const wm_roadgraph *rg, int32_t T, float dt, void *ws,
                size_t ws_bytes, wm_tuning *best, void *stream);

/* Kernel timing, a profiling aid (not part of the paper's method).  While
 * enabled (process-wide), wm_rollout, wm_rollout_backward, wm_observe
 * and wm_offroad bracket their main kernel with HIP events on the caller's
 * stream.  wm_profile_collect waits for the recorded events of one entry
 * point (WM_PROF_*), returns the summed kernel time [ms] and the number of
 * launches, and forgets them.  Event pairs are kept for up to 4096 launches
 * per entry point; later launches are not recorded. */
#define WM_PROF_ROLLOUT 0
#define WM_PROF_BACKWARD 1
#define WM_PROF_OBSERVE 2
#define WM_PROF_OFFROAD 3
int wm_profile_enable(int on);
int wm_profile_collect(int which, float *total_ms, int32_t *launches);

/* Static description of a return code. */
const char *wm_error_string(int code);

/* Detail of the last error returned on the calling thread ("" if none). */
const char *wm_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* WM_H */
