/*
 * wm_oracle.c -- plain, slow FP64 reference of the simulator hot path of
 * "Waymax: An Accelerated, Data-Driven Simulator for Large-Scale Autonomous
 * Driving Research" (arXiv 2310.08710).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this library.  It shares no
 * code, header, table or helper with the HIP library; it is written
 * independently from the paper's equations, one object / pair / point at a
 * time, with no blocking, fusion or reordering.
 *
 * All floating point work is IEEE binary64 (the caller widens the float32
 * inputs exactly).  The one exception is the observation's top-k key, which
 * decides an integer result (an index order) and is therefore computed in the
 * kernel's precision, binary32, with a fixed operation order (see or_observe).
 *
 * Conventions (readings of the paper, each restated where it is used):
 *  - state per object: x, y, yaw, vx, vy, length, width, valid (Sec. 3.2 and
 *    App. A.1); length runs along the yaw direction, the box is centred on
 *    (x, y).
 *  - every metric triggers iff its margin is strictly positive.
 *  - "no value" margins are -FLT_MAX (written as a double).
 *  - wrap(a) = a - 2*pi*floor((a + pi) / (2*pi)), in [-pi, pi).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_NO_VALUE (-(double)FLT_MAX)
#define OR_PI 3.14159265358979323846

typedef struct {
    double *x, *y, *yaw, *vx, *vy, *length, *width;
    uint8_t *valid;
} or_state;

typedef struct {
    const double *x, *y, *dir_x, *dir_y;
    const int8_t *type;
    const uint8_t *valid;
} or_roadgraph;

#define OR_ROAD_EDGE 1

static double wrap_angle(double a)
{
    return a - 2.0 * OR_PI * floor((a + OR_PI) / (2.0 * OR_PI));
}

static void copy_object(const or_state *src, int si, or_state *dst, int di)
{
    dst->x[di] = src->x[si];
    dst->y[di] = src->y[si];
    dst->yaw[di] = src->yaw[si];
    dst->vx[di] = src->vx[si];
    dst->vy[di] = src->vy[si];
    dst->length[di] = src->length[si];
    dst->width[di] = src->width[si];
    dst->valid[di] = src->valid[si];
}

/* Offset view of a time-major state sequence: row t of a [T][n] layout. */
static or_state state_row(const or_state *seq, long t, long n)
{
    or_state r;
    r.x = seq->x + t * n;
    r.y = seq->y + t * n;
    r.yaw = seq->yaw + t * n;
    r.vx = seq->vx + t * n;
    r.vy = seq->vy + t * n;
    r.length = seq->length + t * n;
    r.width = seq->width + t * n;
    r.valid = seq->valid + t * n;
    return r;
}

/* ------------------------------------------------------------------------
 * Bicycle forward dynamics, App. A.1 (bicycle action space, forward
 * equations), applied per object, plus the environment's control semantics
 * (Sec. 4.3): objects not selected by the control mask replay the log
 * (next = log_next, including its valid flag); controlled objects that are
 * invalid stay frozen.
 *   v  = sqrt(vx^2 + vy^2)
 *   x' = x + vx dt + a cos(yaw) dt^2 / 2
 *   y' = y + vy dt + a sin(yaw) dt^2 / 2
 *   yaw' = yaw + kappa (v dt + a dt^2 / 2)
 *   v' = v + a dt ;  (vx', vy') = v' (cos yaw', sin yaw')
 * The displacement uses the current yaw even if the velocity is not aligned
 * with it, v' is not clamped, and yaw' is not wrapped (literal reading).
 * ---------------------------------------------------------------------- */
void or_bicycle_forward(int n, const or_state *cur, const double *accel,
                        const double *curvature, const uint8_t *controlled,
                        const or_state *log_next, double dt, or_state *next)
{
    for (int i = 0; i < n; ++i) {
        if (!controlled[i]) {
            copy_object(log_next, i, next, i);
            continue;
        }
        if (!cur->valid[i]) {
            copy_object(cur, i, next, i);
            continue;
        }
        double x = cur->x[i], y = cur->y[i], yaw = cur->yaw[i];
        double vx = cur->vx[i], vy = cur->vy[i];
        double a = accel[i], k = curvature[i];
        double v = sqrt(vx * vx + vy * vy);
        double nx = x + vx * dt + 0.5 * a * cos(yaw) * dt * dt;
        double ny = y + vy * dt + 0.5 * a * sin(yaw) * dt * dt;
        double nyaw = yaw + k * (v * dt + 0.5 * a * dt * dt);
        double nv = v + a * dt;
        next->x[i] = nx;
        next->y[i] = ny;
        next->yaw[i] = nyaw;
        next->vx[i] = nv * cos(nyaw);
        next->vy[i] = nv * sin(nyaw);
        next->length[i] = cur->length[i];
        next->width[i] = cur->width[i];
        next->valid[i] = 1;
    }
}

/* ------------------------------------------------------------------------
 * Bicycle inverse dynamics, App. A.1 (inverse kinematics equation):
 *   a     = (|v'| - |v|) / dt
 *   kappa = (heading(v') - yaw) / (|v| dt + a dt^2 / 2)
 * Readings: the printed heading term arctan(vx'/vy') contradicts the forward
 * equations (vx' = v' cos yaw'); the heading of the velocity vector
 * atan2(vy', vx') is used, and the difference to yaw is wrapped to [-pi, pi).
 * kappa = 0 when the travelled distance is below 1e-6 m.  An action is valid
 * iff both states are valid; otherwise a = kappa = 0.
 * ---------------------------------------------------------------------- */
void or_bicycle_inverse(int n, const or_state *cur, const or_state *nxt, double dt,
                        double *accel, double *curvature, uint8_t *valid)
{
    for (int i = 0; i < n; ++i) {
        if (!(cur->valid[i] && nxt->valid[i])) {
            accel[i] = 0.0;
            curvature[i] = 0.0;
            valid[i] = 0;
            continue;
        }
        double v = sqrt(cur->vx[i] * cur->vx[i] + cur->vy[i] * cur->vy[i]);
        double nv = sqrt(nxt->vx[i] * nxt->vx[i] + nxt->vy[i] * nxt->vy[i]);
        double a = (nv - v) / dt;
        double dist = v * dt + 0.5 * a * dt * dt;
        double heading = atan2(nxt->vy[i], nxt->vx[i]);
        double k = fabs(dist) < 1e-6 ? 0.0 : wrap_angle(heading - cur->yaw[i]) / dist;
        accel[i] = a;
        curvature[i] = k;
        valid[i] = 1;
    }
}

/* ------------------------------------------------------------------------
 * Kinematic infeasibility (Sec. 3.4): the bicycle inverse kinematics of a
 * transition (cur -> nxt) gives (a, kappa); the transition is infeasible when
 * |a| > 6 m/s^2 or |kappa| > 0.3 1/m (strict).  0 unless both states are valid.
 * ---------------------------------------------------------------------- */
void or_infeasibility(int n, const or_state *cur, const or_state *nxt, double dt, uint8_t *out)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *k = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    uint8_t *v = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    or_bicycle_inverse(n, cur, nxt, dt, a, k, v);
    for (int i = 0; i < n; ++i)
        out[i] = (uint8_t)(v[i] && (fabs(a[i]) > 6.0 || fabs(k[i]) > 0.3));
    free(a);
    free(k);
    free(v);
}

/* ------------------------------------------------------------------------
 * Delta action space, App. A.1 (delta forward and inverse equations):
 *   x' = x + dx, y' = y + dy, yaw' = yaw + dyaw,
 *   vx' = (x' - x)/dt, vy' = (y' - y)/dt;   inverse: d = s' - s.
 * Same control semantics as the bicycle model.
 * ---------------------------------------------------------------------- */
void or_delta_forward(int n, const or_state *cur, const double *dx, const double *dy,
                      const double *dyaw, const uint8_t *controlled,
                      const or_state *log_next, double dt, or_state *next)
{
    for (int i = 0; i < n; ++i) {
        if (!controlled[i]) {
            copy_object(log_next, i, next, i);
            continue;
        }
        if (!cur->valid[i]) {
            copy_object(cur, i, next, i);
            continue;
        }
        double nx = cur->x[i] + dx[i];
        double ny = cur->y[i] + dy[i];
        next->x[i] = nx;
        next->y[i] = ny;
        next->yaw[i] = cur->yaw[i] + dyaw[i];
        next->vx[i] = (nx - cur->x[i]) / dt;
        next->vy[i] = (ny - cur->y[i]) / dt;
        next->length[i] = cur->length[i];
        next->width[i] = cur->width[i];
        next->valid[i] = 1;
    }
}

void or_delta_inverse(int n, const or_state *cur, const or_state *nxt,
                      double *dx, double *dy, double *dyaw, uint8_t *valid)
{
    for (int i = 0; i < n; ++i) {
        int ok = cur->valid[i] && nxt->valid[i];
        dx[i] = ok ? nxt->x[i] - cur->x[i] : 0.0;
        dy[i] = ok ? nxt->y[i] - cur->y[i] : 0.0;
        dyaw[i] = ok ? nxt->yaw[i] - cur->yaw[i] : 0.0;
        valid[i] = (uint8_t)ok;
    }
}

/* ------------------------------------------------------------------------
 * Discretized actions (Sec. 5.2, Expert: "the inverse is computed by
 * discretizing the continuous inverse").  Reading: `bins` values evenly
 * spaced over [lo, hi] (bins >= 2); each value maps to the nearest one, a
 * value half-way between two goes to the upper one, values outside the range
 * to the end bins.  The index is an integer decided by floating point, so it
 * is computed in the kernel's precision (binary32) with a fixed operation
 * order: u = (v - lo) * ((bins - 1) / (hi - lo)), index = floor(u + 0.5).
 * ---------------------------------------------------------------------- */
void or_discretize(int n, const float *values, float lo, float hi, int bins, int32_t *index, float *snapped)
{
    volatile float scale = (float)(bins - 1) / (hi - lo);
    volatile float step = (hi - lo) / (float)(bins - 1);
    for (int i = 0; i < n; ++i) {
        volatile float d = values[i] - lo;
        volatile float u = d * scale;
        volatile float w = u + 0.5f;
        int k;
        if (!(w >= 0.0f))
            k = 0;
        else if (w >= (float)bins)
            k = bins - 1;
        else
            k = (int)floorf(w);
        if (k > bins - 1)
            k = bins - 1;
        if (k < 0)
            k = 0;
        index[i] = k;
        if (snapped) {
            volatile float kv = (float)k * step;
            snapped[i] = lo + kv;
        }
    }
}

/* ------------------------------------------------------------------------
 * Collision (Sec. 3.4, Collision): two objects collide when their 2D
 * top-down boxes overlap.  For two rectangles the separating-axis theorem
 * makes that exact: they overlap iff their projections overlap on all four
 * face normals u_a, w_a, u_b, w_b (u = heading, w = left).  The overlap
 * margin is the smallest projection overlap
 *   g(axis) = r_a(axis) + r_b(axis) - |(c_b - c_a) . axis|,
 * r(axis) = half-length |u . axis| + half-width |w . axis|, which is the
 * penetration depth when positive and minus the largest axis gap otherwise.
 * Boxes that only touch do not overlap (strict margin > 0).
 * ---------------------------------------------------------------------- */
static double box_radius(double yaw, double half_len, double half_wid, double ax, double ay)
{
    double ux = cos(yaw), uy = sin(yaw);
    return half_len * fabs(ux * ax + uy * ay) + half_wid * fabs(-uy * ax + ux * ay);
}

double or_sat_margin(double xa, double ya, double yawa, double la, double wa,
                     double xb, double yb, double yawb, double lb, double wb)
{
    double axes[4][2] = {
        {cos(yawa), sin(yawa)}, {-sin(yawa), cos(yawa)},
        {cos(yawb), sin(yawb)}, {-sin(yawb), cos(yawb)},
    };
    double dx = xb - xa, dy = yb - ya;
    double m = 0.0;
    for (int k = 0; k < 4; ++k) {
        double ax = axes[k][0], ay = axes[k][1];
        double g = box_radius(yawa, 0.5 * la, 0.5 * wa, ax, ay)
                 + box_radius(yawb, 0.5 * lb, 0.5 * wb, ax, ay)
                 - fabs(dx * ax + dy * ay);
        if (k == 0 || g < m)
            m = g;
    }
    return m;
}

/* Per scenario s with N_s objects: optional full margin matrix (row-major
 * N_s x N_s block at offset sum_{s'<s} N_s'^2; diagonal and pairs with an
 * invalid object are -FLT_MAX), per-object max margin over partners and the
 * collision flag max margin > 0. */
void or_overlap(int S, const int32_t *obj_off, const or_state *st,
                double *pair_margin, uint8_t *collision, double *max_margin)
{
    long block = 0;
    for (int s = 0; s < S; ++s) {
        int o = obj_off[s], N = obj_off[s + 1] - obj_off[s];
        for (int i = 0; i < N; ++i) {
            double best = OR_NO_VALUE;
            for (int j = 0; j < N; ++j) {
                double m = OR_NO_VALUE;
                int a = o + i, b = o + j;
                if (i != j && st->valid[a] && st->valid[b])
                    m = or_sat_margin(st->x[a], st->y[a], st->yaw[a], st->length[a], st->width[a],
                                      st->x[b], st->y[b], st->yaw[b], st->length[b], st->width[b]);
                if (pair_margin)
                    pair_margin[block + (long)i * N + j] = m;
                if (m > best)
                    best = m;
            }
            if (max_margin)
                max_margin[o + i] = best;
            if (collision)
                collision[o + i] = (uint8_t)(best > 0.0);
        }
        block += (long)N * N;
    }
}

/* ------------------------------------------------------------------------
 * Off-road (Sec. 3.4, Off-Road): a vehicle is on the road when it is on the
 * left of the oriented road edge, off the road otherwise.  Readings:
 *  - the test is applied to each of the four box corners, in the order
 *    front-left, front-right, rear-right, rear-left
 *    (c + l u + h w, c + l u - h w, c - l u - h w, c - l u + h w);
 *  - the reference edge point of a corner is the nearest valid point of type
 *    road edge (2D Euclidean distance; ties go to the lowest index);
 *  - side: s = -cross(dir, corner - q) is positive on the right (off road);
 *    s == 0 counts as on the road;
 *  - object margin = max over corners of s; offroad iff margin > 0; with no
 *    edge point the margin is -FLT_MAX and the object is on the road.
 * Near-tie report: a corner is ambiguous when |s| < band, or when another
 * edge point lies within `band` metres of the nearest distance and falls on
 * the other side (the mask may flip); it is tied when another edge point lies
 * within `band` metres of the nearest distance at all (the nearest index and
 * the margin may change, the side need not).  `nearest` holds scenario-local
 * point indices (-1: none).
 * ---------------------------------------------------------------------- */
void or_offroad(int S, const int32_t *obj_off, const int32_t *rg_off, const or_state *st,
                const or_roadgraph *rg, double band, double *margin, uint8_t *offroad,
                int32_t *nearest, double *corner_margin, uint8_t *corner_ambiguous, uint8_t *corner_tied)
{
    static const double sl[4] = {1.0, 1.0, -1.0, -1.0};
    static const double sw[4] = {1.0, -1.0, -1.0, 1.0};
    for (int s = 0; s < S; ++s) {
        int p0 = rg_off[s], P = rg_off[s + 1] - rg_off[s];
        for (int i = obj_off[s]; i < obj_off[s + 1]; ++i) {
            double best_margin = OR_NO_VALUE;
            for (int k = 0; k < 4; ++k) {
                int q = -1;
                double qd = 0.0, sk = OR_NO_VALUE;
                int amb = 0, tied = 0;
                if (st->valid[i]) {
                    double c = cos(st->yaw[i]), sn = sin(st->yaw[i]);
                    double hl = 0.5 * st->length[i], hw = 0.5 * st->width[i];
                    double cx = st->x[i] + sl[k] * hl * c - sw[k] * hw * sn;
                    double cy = st->y[i] + sl[k] * hl * sn + sw[k] * hw * c;
                    for (int j = 0; j < P; ++j) {
                        int g = p0 + j;
                        if (!rg->valid[g] || rg->type[g] != OR_ROAD_EDGE)
                            continue;
                        double d = sqrt((cx - rg->x[g]) * (cx - rg->x[g]) + (cy - rg->y[g]) * (cy - rg->y[g]));
                        if (q < 0 || d < qd) {
                            q = j;
                            qd = d;
                        }
                    }
                    if (q >= 0) {
                        int g = p0 + q;
                        sk = -(rg->dir_x[g] * (cy - rg->y[g]) - rg->dir_y[g] * (cx - rg->x[g]));
                        amb = fabs(sk) < band;
                        for (int j = 0; j < P && !(amb && tied); ++j) {
                            int h = p0 + j;
                            if (j == q || !rg->valid[h] || rg->type[h] != OR_ROAD_EDGE)
                                continue;
                            double d = sqrt((cx - rg->x[h]) * (cx - rg->x[h]) + (cy - rg->y[h]) * (cy - rg->y[h]));
                            if (d <= qd + band) {
                                double sj = -(rg->dir_x[h] * (cy - rg->y[h]) - rg->dir_y[h] * (cx - rg->x[h]));
                                tied = 1;
                                if ((sj > 0.0) != (sk > 0.0))
                                    amb = 1;
                            }
                        }
                    }
                }
                if (nearest)
                    nearest[4L * i + k] = q;
                if (corner_margin)
                    corner_margin[4L * i + k] = sk;
                if (corner_ambiguous)
                    corner_ambiguous[4L * i + k] = (uint8_t)amb;
                if (corner_tied)
                    corner_tied[4L * i + k] = (uint8_t)tied;
                if (sk > best_margin)
                    best_margin = sk;
            }
            if (margin)
                margin[i] = best_margin;
            if (offroad)
                offroad[i] = (uint8_t)(best_margin > 0.0);
        }
    }
}

/* ------------------------------------------------------------------------
 * Displacement error (Sec. 3.4, Displacement Error): L2 distance between the
 * simulated and the logged xy at the same step; 0 unless both are valid.
 * (The average over steps is taken by the caller over valid entries.)
 * ---------------------------------------------------------------------- */
void or_log_divergence(int n, const or_state *sim, const or_state *log, double *out)
{
    for (int i = 0; i < n; ++i) {
        if (sim->valid[i] && log->valid[i]) {
            double dx = sim->x[i] - log->x[i], dy = sim->y[i] - log->y[i];
            out[i] = sqrt(dx * dx + dy * dy);
        } else {
            out[i] = 0.0;
        }
    }
}

/* ------------------------------------------------------------------------
 * Default observation (Sec. 3.2): other objects moved into the agent's own
 * frame, and the road graph sub-sampled by distance.  Readings: the sample is
 * the k nearest valid points (any type) to the ego centre, sorted by
 * (distance, index), padded with -1; features are
 *   objects: R(-yaw_e)(p - p_e), wrap(yaw - yaw_e), R(-yaw_e) v, length,
 *            width, valid   (8 floats; invalid or padded slots are 0)
 *   points:  R(-yaw_e)(q - p_e), R(-yaw_e) dir          (4 floats, pad 0)
 * The point order is an integer decision, so its key is taken in the
 * kernel's precision: key = fl32(fl32(dx*dx) + fl32(dy*dy)) with
 * dx = fl32(qx - ex), dy = fl32(qy - ey), no fused multiply-add.  Selection is
 * k passes of "smallest (key, index) above the previous one".
 * Indices are scenario-local.  An invalid ego yields -1 / zeros.
 * ---------------------------------------------------------------------- */
static float topk_key(double qx, double qy, double ex, double ey)
{
    volatile float dx = (float)qx - (float)ex;
    volatile float dy = (float)qy - (float)ey;
    volatile float xx = dx * dx;
    volatile float yy = dy * dy;
    volatile float d2 = xx + yy;
    return d2;
}

void or_observe(int S, const int32_t *obj_off, const int32_t *rg_off, const or_state *st,
                const or_roadgraph *rg, const int32_t *ego, int E, int k, int max_objects,
                int32_t *rg_idx, double *rg_feat, double *obj_feat)
{
    for (int s = 0; s < S; ++s) {
        int o = obj_off[s], N = obj_off[s + 1] - obj_off[s];
        int p0 = rg_off[s], P = rg_off[s + 1] - rg_off[s];
        for (int e = 0; e < E; ++e) {
            long slot = (long)s * E + e;
            int g = ego[slot];
            int32_t *idx = rg_idx + slot * k;
            double *rf = rg_feat ? rg_feat + slot * k * 4 : NULL;
            double *of = obj_feat ? obj_feat + slot * (long)max_objects * 8 : NULL;
            for (int r = 0; r < k; ++r) {
                idx[r] = -1;
                if (rf)
                    rf[4 * r] = rf[4 * r + 1] = rf[4 * r + 2] = rf[4 * r + 3] = 0.0;
            }
            if (of)
                for (long r = 0; r < (long)max_objects * 8; ++r)
                    of[r] = 0.0;
            if (!st->valid[g])
                continue;
            double ex = st->x[g], ey = st->y[g], eyaw = st->yaw[g];
            double c = cos(eyaw), sn = sin(eyaw);
            if (of) {
                for (int j = 0; j < N; ++j) {
                    int h = o + j;
                    if (!st->valid[h])
                        continue;
                    double dx = st->x[h] - ex, dy = st->y[h] - ey;
                    double *f = of + 8L * j;
                    f[0] = c * dx + sn * dy;
                    f[1] = -sn * dx + c * dy;
                    f[2] = wrap_angle(st->yaw[h] - eyaw);
                    f[3] = c * st->vx[h] + sn * st->vy[h];
                    f[4] = -sn * st->vx[h] + c * st->vy[h];
                    f[5] = st->length[h];
                    f[6] = st->width[h];
                    f[7] = 1.0;
                }
            }
            float prev_key = 0.0f;
            int prev_idx = -1;
            for (int r = 0; r < k; ++r) {
                int bj = -1;
                float bkey = 0.0f;
                for (int j = 0; j < P; ++j) {
                    if (!rg->valid[p0 + j])
                        continue;
                    float key = topk_key(rg->x[p0 + j], rg->y[p0 + j], ex, ey);
                    int after_prev = prev_idx < 0 || key > prev_key || (key == prev_key && j > prev_idx);
                    if (!after_prev)
                        continue;
                    if (bj < 0 || key < bkey || (key == bkey && j < bj)) {
                        bj = j;
                        bkey = key;
                    }
                }
                if (bj < 0)
                    break;
                idx[r] = bj;
                prev_idx = bj;
                prev_key = bkey;
                if (rf) {
                    int h = p0 + bj;
                    double dx = rg->x[h] - ex, dy = rg->y[h] - ey;
                    rf[4 * r + 0] = c * dx + sn * dy;
                    rf[4 * r + 1] = -sn * dx + c * dy;
                    rf[4 * r + 2] = c * rg->dir_x[h] + sn * rg->dir_y[h];
                    rf[4 * r + 3] = -sn * rg->dir_x[h] + c * rg->dir_y[h];
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------
 * Training loss used for the differentiable rollout (the paper's
 * differentiable-simulation claim, Sec. 1 and Sec. 6; the loss itself is a
 * reading): per scenario and step t = 1..T
 *   sum over controlled objects valid in sim and log of |p - p_log|^2
 * + sum over unordered pairs (i < j), both valid, at least one controlled, of
 *   sigmoid(margin_ij / 0.1 m).
 * ---------------------------------------------------------------------- */
#define OR_SOFT_SCALE 0.1

static double sigmoid(double z)
{
    return 1.0 / (1.0 + exp(-z));
}

static double step_loss(int o, int N, const or_state *st, const or_state *log, const uint8_t *controlled)
{
    double L = 0.0;
    for (int i = o; i < o + N; ++i) {
        if (controlled[i] && st->valid[i] && log->valid[i]) {
            double dx = st->x[i] - log->x[i], dy = st->y[i] - log->y[i];
            L += dx * dx + dy * dy;
        }
    }
    for (int i = o; i < o + N; ++i)
        for (int j = i + 1; j < o + N; ++j) {
            if (!(st->valid[i] && st->valid[j]) || !(controlled[i] || controlled[j]))
                continue;
            double m = or_sat_margin(st->x[i], st->y[i], st->yaw[i], st->length[i], st->width[i],
                                     st->x[j], st->y[j], st->yaw[j], st->length[j], st->width[j]);
            L += sigmoid(m / OR_SOFT_SCALE);
        }
    return L;
}

/* Loss terms of one state against its log, per scenario (loss[S]). */
void or_state_loss(int S, const int32_t *obj_off, const or_state *st, const or_state *log,
                   const uint8_t *controlled, double *loss)
{
    for (int s = 0; s < S; ++s)
        loss[s] = step_loss(obj_off[s], obj_off[s + 1] - obj_off[s], st, log, controlled);
}

/* ------------------------------------------------------------------------
 * Rollout (Sec. 5.1, Rollout; Sec. 4.1 step): starting from init (the state
 * at the current time), for t = 1..T
 *   state_t = step(state_{t-1}, action_t, log_t)
 * and the metrics are evaluated on the successor state state_t against
 * log_t.  Sequences are time-major: actions [T][n], logs [T+1][n] with row 0
 * at the initial time, trajectory and metrics [T][n].  Any output may be
 * NULL.  loss [S] follows step_loss summed over t.
 * ---------------------------------------------------------------------- */
void or_rollout(int S, const int32_t *obj_off, const int32_t *rg_off, const or_state *init,
                const double *accel, const double *curvature, const uint8_t *controlled,
                const or_state *log_seq, const or_roadgraph *rg, int T, double dt,
                or_state *traj, uint8_t *collision, double *overlap_margin,
                uint8_t *offroad, double *offroad_margin, double *log_div, double *loss)
{
    long n = obj_off[S];
    double *buf = (double *)malloc(sizeof(double) * 14 * n);
    uint8_t *vbuf = (uint8_t *)malloc(2 * n);
    or_state a = {buf, buf + n, buf + 2 * n, buf + 3 * n, buf + 4 * n, buf + 5 * n, buf + 6 * n, vbuf};
    or_state b = {buf + 7 * n, buf + 8 * n, buf + 9 * n, buf + 10 * n, buf + 11 * n, buf + 12 * n,
                  buf + 13 * n, vbuf + n};
    for (long i = 0; i < n; ++i)
        copy_object(init, (int)i, &a, (int)i);
    if (loss)
        for (int s = 0; s < S; ++s)
            loss[s] = 0.0;
    or_state *cur = &a, *nxt = &b;
    for (int t = 1; t <= T; ++t) {
        or_state lg = state_row(log_seq, t, n);
        or_bicycle_forward((int)n, cur, accel + (t - 1) * n, curvature + (t - 1) * n, controlled, &lg, dt, nxt);
        long row = (long)(t - 1) * n;
        if (traj) {
            or_state tr = state_row(traj, t - 1, n);
            for (long i = 0; i < n; ++i)
                copy_object(nxt, (int)i, &tr, (int)i);
        }
        or_overlap(S, obj_off, nxt, NULL, collision ? collision + row : NULL,
                   overlap_margin ? overlap_margin + row : NULL);
        if (rg && (offroad || offroad_margin))
            or_offroad(S, obj_off, rg_off, nxt, rg, 0.0, offroad_margin ? offroad_margin + row : NULL,
                       offroad ? offroad + row : NULL, NULL, NULL, NULL, NULL);
        if (log_div)
            or_log_divergence((int)n, nxt, &lg, log_div + row);
        if (loss)
            for (int s = 0; s < S; ++s)
                loss[s] += step_loss(obj_off[s], obj_off[s + 1] - obj_off[s], nxt, &lg, controlled);
        or_state *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    free(buf);
    free(vbuf);
}

/* Loss only (no metrics outputs), for finite differences. */
void or_rollout_loss(int S, const int32_t *obj_off, const or_state *init, const double *accel,
                     const double *curvature, const uint8_t *controlled, const or_state *log_seq,
                     int T, double dt, double *loss)
{
    or_rollout(S, obj_off, NULL, init, accel, curvature, controlled, log_seq, NULL, T, dt,
               NULL, NULL, NULL, NULL, NULL, NULL, loss);
}

/* ------------------------------------------------------------------------
 * IDM sim agents (Sec. 3.5, simulated agent behaviour): uncontrolled objects
 * follow their logged path with a speed from the intelligent driver model
 * (Treiber, Hennecke and Helbing, 2000).  The paper gives no parameters or
 * procedure beyond that, so every step below is a reading:
 *  - an IDM agent is an uncontrolled object that is valid in every row
 *    0..T of the log window; every other uncontrolled object replays the
 *    log.  Its path is the polyline of its logged positions, rows 0..T, with
 *    cumulative arc length L_0 = 0, L_k = L_{k-1} + |P_k - P_{k-1}|; its
 *    progress sigma starts at 0 (row 0 is the initial state).
 *  - pose at progress s: with k the first row having L_k > s, the position
 *    interpolated linearly between rows k-1 and k at lambda =
 *    (s - L_{k-1}) / (L_k - L_{k-1}) and the yaw yaw_{k-1} + lambda *
 *    wrap(yaw_k - yaw_{k-1}); with no such row, row T's position and yaw.
 *  - lead: lookahead poses at s_m = sigma + m * step, m = 1..M, while
 *    s_m <= L_T, each carrying the agent's box; the lead is the other valid
 *    object whose current box overlaps (separating-axis margin > 0) the pose
 *    with the smallest m, then the lowest index; the gap is (m - 1) * step
 *    and the lead's speed is its velocity projected on the agent's yaw.
 *  - acceleration, with v = |(vx, vy)|:
 *      a = a_max (1 - (v / v0)^delta - (s* / gap)^2),
 *      s* = s0 + max(0, v T_h + v (v - v_lead) / (2 sqrt(a_max b))),
 *    without the interaction term when there is no lead, a = -brake when the
 *    gap is 0, and a clamped to [-brake, a_max].
 *  - motion: v' = v + a dt and advance v dt + a dt^2 / 2; if v' < 0 the
 *    agent stops within the step: advance v^2 / (2 |a|), v' = 0.  An agent
 *    that reaches the end of its path halts there: sigma' = L_T, v' = 0;
 *    otherwise sigma' = sigma + advance.  The next state is the pose at
 *    sigma' with velocity v' along its yaw, and length, width and valid of
 *    log row t.
 *  - the decision margin of an agent's step is the smallest of the
 *    |separating-axis margins| of the tests that decide the lead (all objects
 *    at poses 1..m of the lead, all poses without a lead) and, when the
 *    halt would change the speed (v' > 0), the distance |L_T - (sigma +
 *    advance)| that decides the halt at the path end.
 * ---------------------------------------------------------------------- */
typedef struct {
    double v0, s0, headway, a_max, b_comf, delta, brake, step;
    int poses;
} or_idm;

static void idm_pose(long i, int T, long n, const or_state *log, const double *L, double s, double *px,
                     double *py, double *pyaw)
{
    int k = 1;
    while (k <= T && !(L[k] > s))
        ++k;
    if (k > T) {
        *px = log->x[(long)T * n + i];
        *py = log->y[(long)T * n + i];
        *pyaw = log->yaw[(long)T * n + i];
        return;
    }
    long a = (long)(k - 1) * n + i, b = (long)k * n + i;
    double lam = (s - L[k - 1]) / (L[k] - L[k - 1]);
    *px = log->x[a] + lam * (log->x[b] - log->x[a]);
    *py = log->y[a] + lam * (log->y[b] - log->y[a]);
    *pyaw = log->yaw[a] + lam * wrap_angle(log->yaw[b] - log->yaw[a]);
}

/* One IDM step of agent i of scenario [o0, o1) from state cur (all objects
 * at time t-1); writes row t of the next state into nxt and returns the
 * decision margin. */
static double idm_step(long i, long o0, long o1, int T, long n, const or_state *cur, const or_state *log_seq,
                       const double *L, double *sigma, const or_idm *p, double dt, int t, or_state *nxt)
{
    double minabs = INFINITY;
    int lead = -1;
    double gap = 0.0;
    for (int m = 1; m <= p->poses && lead < 0; ++m) {
        double sm = sigma[i] + m * p->step;
        if (sm > L[T])
            break;
        double px, py, pyaw;
        idm_pose(i, T, n, log_seq, L, sm, &px, &py, &pyaw);
        for (long j = o0; j < o1; ++j) {
            if (j == i || !cur->valid[j])
                continue;
            double g = or_sat_margin(px, py, pyaw, cur->length[i], cur->width[i], cur->x[j], cur->y[j],
                                     cur->yaw[j], cur->length[j], cur->width[j]);
            if (fabs(g) < minabs)
                minabs = fabs(g);
            if (g > 0.0 && lead < 0) {
                lead = (int)j;
                gap = (m - 1) * p->step;
            }
        }
    }
    double v = sqrt(cur->vx[i] * cur->vx[i] + cur->vy[i] * cur->vy[i]);
    double a = p->a_max * (1.0 - pow(v / p->v0, p->delta));
    if (lead >= 0) {
        double vl = cur->vx[lead] * cos(cur->yaw[i]) + cur->vy[lead] * sin(cur->yaw[i]);
        double ss = p->s0 + fmax(0.0, v * p->headway + v * (v - vl) / (2.0 * sqrt(p->a_max * p->b_comf)));
        a = gap > 0.0 ? a - p->a_max * (ss / gap) * (ss / gap) : -p->brake;
    }
    a = fmin(fmax(a, -p->brake), p->a_max);
    double vn = v + a * dt, adv;
    if (vn >= 0.0) {
        adv = v * dt + 0.5 * a * dt * dt;
    } else {
        adv = v * v / (2.0 * -a);
        vn = 0.0;
    }
    if (vn > 0.0 && fabs(L[T] - (sigma[i] + adv)) < minabs)
        minabs = fabs(L[T] - (sigma[i] + adv));
    if (sigma[i] + adv >= L[T]) {
        sigma[i] = L[T];
        vn = 0.0;
    } else {
        sigma[i] += adv;
    }
    double x, y, yaw;
    idm_pose(i, T, n, log_seq, L, sigma[i], &x, &y, &yaw);
    long r = (long)t * n + i;
    nxt->x[i] = x;
    nxt->y[i] = y;
    nxt->yaw[i] = yaw;
    nxt->vx[i] = vn * cos(yaw);
    nxt->vy[i] = vn * sin(yaw);
    nxt->length[i] = log_seq->length[r];
    nxt->width[i] = log_seq->width[r];
    nxt->valid[i] = log_seq->valid[r];
    return minabs;
}

/* Rollout as or_rollout (no loss) with the uncontrolled objects that have a
 * fully valid log window driven by IDM.  `margin` [T][n] (optional) receives
 * each IDM agent's decision margin per step (+inf for other objects). */
void or_rollout_idm(int S, const int32_t *obj_off, const int32_t *rg_off, const or_state *init,
                    const double *accel, const double *curvature, const uint8_t *controlled,
                    const or_state *log_seq, const or_roadgraph *rg, int T, double dt, const or_idm *p,
                    or_state *traj, uint8_t *collision, double *overlap_margin, uint8_t *offroad,
                    double *offroad_margin, double *log_div, double *margin)
{
    long n = obj_off[S];
    double *buf = (double *)malloc(sizeof(double) * 14 * n);
    uint8_t *vbuf = (uint8_t *)malloc(2 * n);
    double *L = (double *)malloc(sizeof(double) * (size_t)(T + 1) * (size_t)(n > 0 ? n : 1));
    double *sigma = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    uint8_t *agent = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    or_state a = {buf, buf + n, buf + 2 * n, buf + 3 * n, buf + 4 * n, buf + 5 * n, buf + 6 * n, vbuf};
    or_state b = {buf + 7 * n, buf + 8 * n, buf + 9 * n, buf + 10 * n, buf + 11 * n, buf + 12 * n,
                  buf + 13 * n, vbuf + n};
    for (long i = 0; i < n; ++i) {
        copy_object(init, (int)i, &a, (int)i);
        int ok = !controlled[i];
        for (int k = 0; k <= T && ok; ++k)
            ok = log_seq->valid[(long)k * n + i] != 0;
        agent[i] = (uint8_t)ok;
        double *Li = L + (size_t)i * (T + 1);
        Li[0] = 0.0;
        for (int k = 1; k <= T; ++k) {
            long r0 = (long)(k - 1) * n + i, r1 = (long)k * n + i;
            Li[k] = Li[k - 1] + sqrt((log_seq->x[r1] - log_seq->x[r0]) * (log_seq->x[r1] - log_seq->x[r0]) +
                                     (log_seq->y[r1] - log_seq->y[r0]) * (log_seq->y[r1] - log_seq->y[r0]));
        }
    }
    or_state *cur = &a, *nxt = &b;
    for (int t = 1; t <= T; ++t) {
        or_state lg = state_row(log_seq, t, n);
        long row = (long)(t - 1) * n;
        or_bicycle_forward((int)n, cur, accel + (t - 1) * n, curvature + (t - 1) * n, controlled, &lg, dt, nxt);
        for (int s = 0; s < S; ++s)
            for (long i = obj_off[s]; i < obj_off[s + 1]; ++i) {
                double mg = INFINITY;
                if (agent[i])
                    mg = idm_step(i, obj_off[s], obj_off[s + 1], T, n, cur, log_seq, L + (size_t)i * (T + 1),
                                  sigma, p, dt, t, nxt);
                if (margin)
                    margin[row + i] = mg;
            }
        if (traj) {
            or_state tr = state_row(traj, t - 1, n);
            for (long i = 0; i < n; ++i)
                copy_object(nxt, (int)i, &tr, (int)i);
        }
        or_overlap(S, obj_off, nxt, NULL, collision ? collision + row : NULL,
                   overlap_margin ? overlap_margin + row : NULL);
        if (rg && (offroad || offroad_margin))
            or_offroad(S, obj_off, rg_off, nxt, rg, 0.0, offroad_margin ? offroad_margin + row : NULL,
                       offroad ? offroad + row : NULL, NULL, NULL, NULL, NULL);
        if (log_div)
            or_log_divergence((int)n, nxt, &lg, log_div + row);
        or_state *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    free(buf);
    free(vbuf);
    free(L);
    free(sigma);
    free(agent);
}

/* ------------------------------------------------------------------------
 * Reverse-mode gradient of the rollout loss with respect to the actions,
 * by hand, with the whole forward trajectory kept (no checkpointing).
 * Conventions at non-smooth points: sgn(0) = +1 for |.|; the lowest axis
 * index wins a tie of the separating-axis minimum; d|v|/d(vx, vy) = 0 at
 * v = 0.  Gradients of uncontrolled or invalid objects are zero.  dloss[s]
 * scales scenario s.
 * ---------------------------------------------------------------------- */
static double sgn1(double u)
{
    return u >= 0.0 ? 1.0 : -1.0;
}

/* Gradient of the separating-axis margin between boxes a and b with respect
 * to (x_a, y_a, yaw_a) and (x_b, y_b, yaw_b).  Axis k: 0 = u_a, 1 = w_a,
 * 2 = u_b, 3 = w_b; g_k = r_a + r_b - |d . axis_k| with d = c_b - c_a. */
static void sat_margin_grad(double xa, double ya, double ta, double la, double wa,
                            double xb, double yb, double tb, double lb, double wb,
                            double ga[3], double gb[3])
{
    double ca = cos(ta), sa = sin(ta), cb = cos(tb), sb = sin(tb);
    double hla = 0.5 * la, hwa = 0.5 * wa, hlb = 0.5 * lb, hwb = 0.5 * wb;
    double dx = xb - xa, dy = yb - ya;
    double delta = tb - ta;
    double cd = cos(delta), sd = sin(delta);
    double C = fabs(cd), Sn = fabs(sd);
    double dC = -sgn1(cd) * sd; /* dC/d(delta) */
    double dS = sgn1(sd) * cd;  /* dS/d(delta) */
    /* projections of d on each axis and their yaw derivatives */
    double pu_a = dx * ca + dy * sa, pw_a = -dx * sa + dy * ca;
    double pu_b = dx * cb + dy * sb, pw_b = -dx * sb + dy * cb;
    double g[4] = {
        hla + hlb * C + hwb * Sn - fabs(pu_a),
        hwa + hlb * Sn + hwb * C - fabs(pw_a),
        hlb + hla * C + hwa * Sn - fabs(pu_b),
        hwb + hla * Sn + hwa * C - fabs(pw_b),
    };
    int k = 0;
    for (int j = 1; j < 4; ++j)
        if (g[j] < g[k])
            k = j;
    double ax, ay, p, rdelta, dp_dta = 0.0, dp_dtb = 0.0;
    switch (k) {
    case 0:
        ax = ca; ay = sa; p = pu_a; rdelta = hlb * dC + hwb * dS; dp_dta = pw_a; break;
    case 1:
        ax = -sa; ay = ca; p = pw_a; rdelta = hlb * dS + hwb * dC; dp_dta = -pu_a; break;
    case 2:
        ax = cb; ay = sb; p = pu_b; rdelta = hla * dC + hwa * dS; dp_dtb = pw_b; break;
    default:
        ax = -sb; ay = cb; p = pw_b; rdelta = hla * dS + hwa * dC; dp_dtb = -pu_b; break;
    }
    double sp = sgn1(p);
    /* g = r(delta) - |p|, d = c_b - c_a, p = d . axis */
    ga[0] = sp * ax;
    ga[1] = sp * ay;
    gb[0] = -sp * ax;
    gb[1] = -sp * ay;
    ga[2] = -rdelta - sp * dp_dta;
    gb[2] = rdelta - sp * dp_dtb;
}

void or_rollout_grad(int S, const int32_t *obj_off, const or_state *init, const double *accel,
                     const double *curvature, const uint8_t *controlled, const or_state *log_seq,
                     int T, double dt, const double *dloss, double *grad_accel,
                     double *grad_curvature, double *loss)
{
    long n = obj_off[S];
    /* tape: states 0..T */
    double *tape = (double *)malloc(sizeof(double) * 7 * n * (T + 1));
    uint8_t *vt = (uint8_t *)malloc((size_t)n * (T + 1));
    or_state seq = {tape, tape + n * (T + 1), tape + 2 * n * (T + 1), tape + 3 * n * (T + 1),
                    tape + 4 * n * (T + 1), tape + 5 * n * (T + 1), tape + 6 * n * (T + 1), vt};
    or_state s0 = state_row(&seq, 0, n);
    for (long i = 0; i < n; ++i)
        copy_object(init, (int)i, &s0, (int)i);
    for (int t = 1; t <= T; ++t) {
        or_state prev = state_row(&seq, t - 1, n), now = state_row(&seq, t, n);
        or_state lg = state_row(log_seq, t, n);
        or_bicycle_forward((int)n, &prev, accel + (t - 1) * n, curvature + (t - 1) * n, controlled, &lg, dt, &now);
    }
    if (loss) {
        for (int s = 0; s < S; ++s) {
            loss[s] = 0.0;
            for (int t = 1; t <= T; ++t) {
                or_state now = state_row(&seq, t, n), lg = state_row(log_seq, t, n);
                loss[s] += step_loss(obj_off[s], obj_off[s + 1] - obj_off[s], &now, &lg, controlled);
            }
        }
    }
    /* adjoints of (x, y, yaw, vx, vy) of the state being processed */
    double *adj = (double *)calloc((size_t)5 * n, sizeof(double));
    for (long i = 0; i < n * T; ++i) {
        grad_accel[i] = 0.0;
        grad_curvature[i] = 0.0;
    }
    for (int t = T; t >= 1; --t) {
        or_state now = state_row(&seq, t, n), prev = state_row(&seq, t - 1, n);
        or_state lg = state_row(log_seq, t, n);
        /* loss terms at step t */
        for (int s = 0; s < S; ++s) {
            double w = dloss[s];
            int o = obj_off[s], N = obj_off[s + 1] - obj_off[s];
            for (int i = o; i < o + N; ++i) {
                if (controlled[i] && now.valid[i] && lg.valid[i]) {
                    adj[5 * i + 0] += w * 2.0 * (now.x[i] - lg.x[i]);
                    adj[5 * i + 1] += w * 2.0 * (now.y[i] - lg.y[i]);
                }
            }
            for (int i = o; i < o + N; ++i)
                for (int j = i + 1; j < o + N; ++j) {
                    if (!(now.valid[i] && now.valid[j]) || !(controlled[i] || controlled[j]))
                        continue;
                    double m = or_sat_margin(now.x[i], now.y[i], now.yaw[i], now.length[i], now.width[i],
                                             now.x[j], now.y[j], now.yaw[j], now.length[j], now.width[j]);
                    double sg = sigmoid(m / OR_SOFT_SCALE);
                    double dm = w * sg * (1.0 - sg) / OR_SOFT_SCALE;
                    double ga[3], gb[3];
                    sat_margin_grad(now.x[i], now.y[i], now.yaw[i], now.length[i], now.width[i],
                                    now.x[j], now.y[j], now.yaw[j], now.length[j], now.width[j], ga, gb);
                    for (int c = 0; c < 3; ++c) {
                        adj[5 * i + c] += dm * ga[c];
                        adj[5 * j + c] += dm * gb[c];
                    }
                }
        }
        /* back through the dynamics of step t */
        for (long i = 0; i < n; ++i) {
            double *ad = adj + 5 * i;
            if (!controlled[i] || !prev.valid[i]) {
                /* replayed from the log or frozen: no dependence on actions,
                   and a replayed state does not depend on the previous one */
                if (!controlled[i])
                    ad[0] = ad[1] = ad[2] = ad[3] = ad[4] = 0.0;
                continue;
            }
            double yaw = prev.yaw[i], vx = prev.vx[i], vy = prev.vy[i];
            double a = accel[(t - 1) * n + i], k = curvature[(t - 1) * n + i];
            double v = sqrt(vx * vx + vy * vy);
            double D = v * dt + 0.5 * a * dt * dt;
            double nyaw = now.yaw[i];
            double nv = v + a * dt;
            double bx = ad[0], by = ad[1], byaw = ad[2], bvx = ad[3], bvy = ad[4];
            double bnv = bvx * cos(nyaw) + bvy * sin(nyaw);
            double tyaw = byaw + nv * (-bvx * sin(nyaw) + bvy * cos(nyaw));
            double ga = 0.5 * dt * dt * (bx * cos(yaw) + by * sin(yaw) + k * tyaw) + dt * bnv;
            double gk = D * tyaw;
            double pyaw = tyaw + 0.5 * a * dt * dt * (-bx * sin(yaw) + by * cos(yaw));
            double bv = k * dt * tyaw + bnv;
            double pvx = dt * bx + (v > 0.0 ? bv * vx / v : 0.0);
            double pvy = dt * by + (v > 0.0 ? bv * vy / v : 0.0);
            grad_accel[(t - 1) * n + i] = ga;
            grad_curvature[(t - 1) * n + i] = gk;
            ad[0] = bx;
            ad[1] = by;
            ad[2] = pyaw;
            ad[3] = pvx;
            ad[4] = pvy;
        }
    }
    free(adj);
    free(tape);
    free(vt);
}
