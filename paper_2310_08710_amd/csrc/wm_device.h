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

namespace wm {

constexpr int kChunk = 32;            // road-edge points per chunk of the off-road scan
constexpr float kNoValue = -FLT_MAX;  // margin with no defined value
constexpr float kSoftScale = 0.1f;    // soft-overlap scale of the training loss [m]

// Pointer into the constant address space: loads through it whose address is
// wave-uniform become scalar (SMEM) loads that feed VALU ops as SGPR operands.
typedef const float __attribute__((address_space(4))) *uniform_fptr;

// Scenario-major packed state kept in LDS by the fused kernels.
struct ObjLds {
    float *x, *y, *yaw, *vx, *vy, *len, *wid, *c, *s;
    uint8_t *valid, *ctrl;
};

// ---------------------------------------------------------------------------
// Bicycle forward dynamics (App. A.1, forward dynamics equation).
//   v = |(vx, vy)|; x' = x + vx dt + a cos(yaw) dt^2/2; y' likewise with sin;
//   yaw' = yaw + kappa (v dt + a dt^2/2); v' = v + a dt; (vx', vy') = v'(cos, sin)(yaw')
// ---------------------------------------------------------------------------
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

// Gradient of sat_margin with respect to (x, y, yaw) of a and of b, through
// the arg-min axis (lowest axis index on ties), sgn(0) = +1.
__device__ __forceinline__ void sat_margin_grad(const Box &a, const Box &b, float ga[3], float gb[3])
{
    const float dx = b.x - a.x, dy = b.y - a.y;
    const float cd = __builtin_fmaf(a.c, b.c, a.s * b.s);    // cos(delta), delta = yaw_b - yaw_a
    const float sd = __builtin_fmaf(a.c, b.s, -(a.s * b.c)); // sin(delta)
    const float C = fabsf(cd), S = fabsf(sd);
    const float dC = -(cd >= 0.f ? 1.f : -1.f) * sd;
    const float dS = (sd >= 0.f ? 1.f : -1.f) * cd;
    const float pua = __builtin_fmaf(dx, a.c, dy * a.s), pwa = __builtin_fmaf(dy, a.c, -(dx * a.s));
    const float pub = __builtin_fmaf(dx, b.c, dy * b.s), pwb = __builtin_fmaf(dy, b.c, -(dx * b.s));
    const float g[4] = {
        a.hl + __builtin_fmaf(b.hl, C, b.hw * S) - fabsf(pua),
        a.hw + __builtin_fmaf(b.hl, S, b.hw * C) - fabsf(pwa),
        b.hl + __builtin_fmaf(a.hl, C, a.hw * S) - fabsf(pub),
        b.hw + __builtin_fmaf(a.hl, S, a.hw * C) - fabsf(pwb),
    };
    int k = 0;
    if (g[1] < g[k]) k = 1;
    if (g[2] < g[k]) k = 2;
    if (g[3] < g[k]) k = 3;
    float ax, ay, p, rd, dpa = 0.f, dpb = 0.f;
    if (k == 0) {
        ax = a.c; ay = a.s; p = pua; rd = __builtin_fmaf(b.hl, dC, b.hw * dS); dpa = pwa;
    } else if (k == 1) {
        ax = -a.s; ay = a.c; p = pwa; rd = __builtin_fmaf(b.hl, dS, b.hw * dC); dpa = -pua;
    } else if (k == 2) {
        ax = b.c; ay = b.s; p = pub; rd = __builtin_fmaf(a.hl, dC, a.hw * dS); dpb = pwb;
    } else {
        ax = -b.s; ay = b.c; p = pwb; rd = __builtin_fmaf(a.hl, dS, a.hw * dC); dpb = -pub;
    }
    const float sp = p >= 0.f ? 1.f : -1.f;
    ga[0] = sp * ax;
    ga[1] = sp * ay;
    gb[0] = -sp * ax;
    gb[1] = -sp * ay;
    ga[2] = -rd - sp * dpa;
    gb[2] = rd - sp * dpb;
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
// scenario's compacted road-edge list (x, y interleaved; padded with +inf
// points to whole chunks) against R corners held per lane.  The edge address
// is wave-uniform, so every point arrives once per wave through SMEM and is
// used as an SGPR operand by all 64 lanes.  Only the minimum is tracked in the
// inner loop; the first chunk that reaches the final minimum is remembered
// (strict <), and the exact lowest index is recovered later by rescanning that
// one chunk.
// ---------------------------------------------------------------------------
template <int R>
__device__ __forceinline__ void scan_edges(const float *__restrict__ exy, int c0, int c1, const float (&cx)[R],
                                           const float (&cy)[R], float (&best)[R], int (&bchunk)[R])
{
    uniform_fptr e = (uniform_fptr)exy;
    for (int c = c0; c < c1; ++c) {
        float m[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            m[r] = __builtin_inff();
        uniform_fptr p = e + 2 * kChunk * c;
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            const float qx = p[2 * j], qy = p[2 * j + 1];
#pragma unroll
            for (int r = 0; r < R; ++r)
                m[r] = fminf(m[r], edge_d2(qx, qy, cx[r], cy[r]));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (m[r] < best[r]) {
                best[r] = m[r];
                bchunk[r] = c;
            }
        }
    }
}

// Lowest index j in chunk `c` whose distance equals `best` (vector loads).
__device__ __forceinline__ int rescan_chunk(const float2 *__restrict__ exy, int c, float cx, float cy, float best)
{
    const float2 *p = exy + kChunk * c;
    int found = kChunk - 1;   // always inside the chunk, even if no bit-equal match existed
    for (int j = kChunk - 1; j >= 0; --j) {
        const float2 q = p[j];
        if (edge_d2(q.x, q.y, cx, cy) == best)
            found = j;
    }
    return kChunk * c + found;
}

} // namespace wm
