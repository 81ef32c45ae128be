// wm_backward.hip -- hand-written adjoint of the fused rollout's training
// loss with respect to the actions (differentiable simulation, Sec. 1 and
// Sec. 6; dynamics of App. A.1).
//
// One 1024-thread work-group per scenario.  The forward pass stored the state
// every K steps; each segment [cK, min(cK + K, T)] is recomputed from its
// checkpoint with the same device code as the forward (bit-identical states)
// into the workspace and swept in reverse, SB steps at a time:
//   1. every object's state at those SB steps goes to LDS (controlled ones
//      from the recomputation, the others from the log);
//   2. the loss gradient with respect to each controlled object's (x, y,
//      yaw) at each of those steps: sigmoid'(m / 0.1) / 0.1 * dm/d(x, y, yaw)
//      over every pair with a controlled member.  The pair terms do not
//      depend on the adjoint, so all SB steps are done at once: a group of
//      G lanes per (step, controlled object) splits the partners (j = lane,
//      lane + G, ...) and sums them with a fixed shuffle tree.  A lane first
//      marks the partners close enough for a non-zero term (a distance
//      bound); the wave evaluates its marked pairs one per lane, and each
//      lane adds its own terms in ascending partner order;
//   3. one thread per controlled object runs the reverse recursion over the
//      SB steps: the log-divergence term 2 (p - p_log), then back through the
//      bicycle step, with the object's adjoint held in registers.  Its
//      inputs do not depend on the adjoint and are staged in LDS with the
//      states: the log position, and the factors of the step's derivatives
//      that the previous state and the action give (sine and cosine of the
//      previous yaw, speeds, distance, velocity direction), computed in
//      parallel so that the recursion's chain holds no transcendental.
// G depends only on the scenario's object count and SB only changes the
// blocking, so the gradients are identical for every checkpoint interval.
// Only controlled, valid objects carry adjoints: replayed objects do not
// depend on the actions and frozen objects never enter the loss.
#include "wm_device.h"
#include "wm_internal.h"

namespace wm {

constexpr int kBwdThreads = 1024;
constexpr size_t kBwdStageBudget = 128 * 1024;   // LDS for the SB-step blocks
constexpr int kBwdRec = 12;                       // recursion inputs per (step, controlled object)
static_assert(kBwdRec % 4 == 0, "the recursion inputs are read as float4");
// Pair terms whose margin is below -kCullGap are skipped: there -m / kSoftScale
// exceeds 128 / log2(e), the FP32 exponential of the sigmoid overflows to
// infinity and the term is exactly zero.
constexpr float kCullGap = 9.0f;
static_assert(kCullGap / kSoftScale * 1.4426950f > 129.0f, "skipped terms overflow the exponential");
static_assert(WM_MAX_OBJECTS <= 64 * 32, "a lane's partners fit in one 32-bit mask");
constexpr size_t kBwdStepBytes = 16 + 16 + 8 + 3 * 4 + kBwdRec * 4;   // LDS per step and object
static_assert(WM_MAX_OBJECTS <= kBwdThreads, "one thread per controlled object");
static_assert(kBwdStageBudget + (size_t)WM_MAX_OBJECTS * 5 + 16 + (size_t)kBwdThreads / 64 * 64 * (16 + 4) <=
                  160 * 1024,
              "the step blocks, indices, kinds and the per-wave pair lists fit in a CU's LDS");

// Byte offset of the per-wave pair lists in the adjoint's LDS: after the
// step blocks, the controlled indices and the object kinds.
__host__ __device__ constexpr size_t backward_wave_offset(int maxN, int SB)
{
    return ((size_t)SB * maxN * kBwdStepBytes + (size_t)maxN * 5 + 15) / 16 * 16;
}

__device__ __forceinline__ void store_state(float *row, long n, long g, float x, float y, float yaw, float vx, float vy)
{
    row[g] = x;
    row[n + g] = y;
    row[2 * n + g] = yaw;
    row[3 * n + g] = vx;
    row[4 * n + g] = vy;
}

__global__ __launch_bounds__(kBwdThreads) void k_rollout_backward(BackwardArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int maxN = A.maxN, SB = A.SB;
    // LDS: [SB][maxN] (x, y, cos, sin), [SB][maxN] (x, y, reach, 0) for the
    // distance bound (reach: half length + half width + kCullGap), the
    // recursion's inputs [SB][maxN][12] per controlled slot (16-byte
    // aligned), [SB][maxN] (half length or -1 when invalid, half width), the
    // pair-term sums [SB][maxN][3]; the controlled objects' indices; per
    // object 2 (controlled and valid), 1 (controlled, invalid) or 0 (from the
    // log)
    float4 *st4 = (float4 *)smem;
    float4 *tst = st4 + SB * maxN;
    float *rec = (float *)(tst + SB * maxN);
    float2 *st2 = (float2 *)(rec + kBwdRec * SB * maxN);
    float *part = (float *)(st2 + SB * maxN);
    int *cidx = (int *)(part + 3 * SB * maxN);
    uint8_t *kind = (uint8_t *)(cidx + maxN);
    // per wave: the list of marked pairs being evaluated and their terms
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float4 *wres = (float4 *)(smem + backward_wave_offset(maxN, SB)) + 64 * wv;
    int *wslot = (int *)(smem + backward_wave_offset(maxN, SB) + (size_t)kBwdThreads / 64 * 64 * 16) + 64 * wv;
    __shared__ int s_nc;

    const int tid = threadIdx.x, nthr = blockDim.x;
    const int s = blockIdx.x;
    const int o0 = A.obj_off[s], N = A.obj_off[s + 1] - o0;
    const long n = A.n;
    const float w = A.dloss[s];
    const float dt = A.dt, hdt2 = 0.5f * dt * dt;

    if (tid == 0) {
        int nc = 0;
        for (int i = 0; i < N; ++i)
            if (A.act.controlled[o0 + i] && A.init.valid[o0 + i])
                cidx[nc++] = i;
        s_nc = nc;
    }
    for (int i = tid; i < N; i += nthr) {
        const bool ctl = A.act.controlled[o0 + i] != 0, live = ctl && A.init.valid[o0 + i];
        kind[i] = ctl ? (live ? 2 : 1) : 0;
        if (!live)
            for (int t = 0; t < A.T; ++t) {
                A.grad_a[(long)t * n + o0 + i] = 0.f;
                A.grad_k[(long)t * n + o0 + i] = 0.f;
            }
    }
    __syncthreads();
    const int NC = s_nc;
    // partner split: G lanes (a power of two <= 64) per (step, controlled
    // object), about 16 partners each
    int G = 1;
    while (G < 64 && G * 16 < N)
        G <<= 1;
    const int nseg = (A.T + A.K - 1) / A.K;
    float *seg = A.seg;
    // the adjoint of this thread's controlled object (x, y, yaw, vx, vy)
    float bx = 0.f, by = 0.f, byaw = 0.f, bvx = 0.f, bvy = 0.f;
    const int q = tid;
    const int i_own = q < NC ? cidx[q] : 0;
    const long g_own = o0 + i_own;

    for (int c = nseg - 1; c >= 0; --c) {
        const int t0 = c * A.K, t1 = min(A.T, t0 + A.K);
        __syncthreads();   // the previous block's readers of seg are done
        // recompute the controlled objects' states t0..t1 into the workspace,
        // thread q for controlled object q.  The actions go to the (free)
        // block LDS first, RC steps at a time, so that their loads are in
        // flight together rather than one step after another.
        float sx = 0.f, sy = 0.f, syaw = 0.f, svx = 0.f, svy = 0.f;
        if (q < NC) {
            sx = A.ckpt.x[(long)c * n + g_own];
            sy = A.ckpt.y[(long)c * n + g_own];
            syaw = A.ckpt.yaw[(long)c * n + g_own];
            svx = A.ckpt.vx[(long)c * n + g_own];
            svy = A.ckpt.vy[(long)c * n + g_own];
            store_state(seg, n, g_own, sx, sy, syaw, svx, svy);
        }
        float2 *acts = (float2 *)smem;
        const int RC = (int)((size_t)SB * maxN * kBwdStepBytes / sizeof(float2) / max(NC, 1));
        for (int tc = t0; tc < t1; tc += RC) {   // steps tc + 1 .. tc + nr
            const int nr = min(RC, t1 - tc);
            for (int it = tid; it < nr * NC; it += nthr) {
                const int r = it / NC, qq = it - r * NC;
                const long at = (long)(tc + r) * n + o0 + cidx[qq];
                acts[it] = make_float2(A.act.accel[at], A.act.curvature[at]);
            }
            __syncthreads();
            if (q < NC)
                for (int r = 0; r < nr; ++r) {
                    const float2 ak = acts[r * NC + q];
                    bicycle_forward(sx, sy, syaw, svx, svy, ak.x, ak.y, dt);
                    store_state(seg + (long)(tc + r + 1 - t0) * 5 * n, n, g_own, sx, sy, syaw, svx, svy);
                }
            __syncthreads();   // the actions' readers are done, the states are written
        }
        // blocks of SB steps, last block first: steps tb_lo + 1 .. tb_hi
        for (int tb_hi = t1; tb_hi > t0; tb_hi -= SB) {
            const int tb_lo = max(t0, tb_hi - SB), nb = tb_hi - tb_lo;
            // 1. states of every object at steps tb_lo + 1 .. tb_hi (slot tb = t - tb_lo - 1)
            for (int it = tid; it < nb * N; it += nthr) {
                const int tb = it / N, i = it - tb * N;
                const int t = tb_lo + 1 + tb;
                const float *row = seg + (long)(t - t0) * 5 * n;
                const long g = o0 + i, lrow = (long)t * n;
                float x, y, yaw, len, wid;
                uint8_t v;
                const int kd = kind[i];
                if (kd != 0) {
                    v = kd == 2;
                    len = A.init.length[g];
                    wid = A.init.width[g];
                    if (v) {
                        x = row[g];
                        y = row[n + g];
                        yaw = row[2 * n + g];
                    } else {
                        x = A.init.x[g];
                        y = A.init.y[g];
                        yaw = A.init.yaw[g];
                    }
                } else {
                    v = A.log.valid[lrow + g];
                    x = A.log.x[lrow + g];
                    y = A.log.y[lrow + g];
                    yaw = A.log.yaw[lrow + g];
                    len = A.log.length[lrow + g];
                    wid = A.log.width[lrow + g];
                }
                float sn, cs;
                sincosf(yaw, &sn, &cs);
                const int at = tb * maxN + i;
                const float hl = v ? 0.5f * len : -1.f, hw = 0.5f * wid;
                st4[at] = make_float4(x, y, cs, sn);
                tst[at] = make_float4(x, y, hl + hw + kCullGap, 0.f);
                st2[at] = make_float2(hl, hw);
            }
            // the recursion's inputs, which do not depend on the adjoint: the
            // log position at t and the factors of the bicycle step's
            // derivatives that come from the state at t - 1 and the action of
            // step t (computed here, in parallel, off the recursion's chain)
            for (int it = tid; it < nb * NC; it += nthr) {
                const int tb = it / NC, qq = it - tb * NC;
                const int t = tb_lo + 1 + tb;
                const long g = o0 + cidx[qq], lrow = (long)t * n;
                const float *prow = seg + (long)(t - 1 - t0) * 5 * n;
                const float yaw0 = prow[2 * n + g], vx0 = prow[3 * n + g], vy0 = prow[4 * n + g];
                const float a = A.act.accel[(long)(t - 1) * n + g], k = A.act.curvature[(long)(t - 1) * n + g];
                const float v = sqrtf(__builtin_fmaf(vy0, vy0, vx0 * vx0));
                float s0, c0;
                sincosf(yaw0, &s0, &c0);
                float4 *r = (float4 *)(rec + kBwdRec * (tb * maxN + qq));
                r[0] = make_float4(A.log.x[lrow + g], A.log.y[lrow + g], A.log.valid[lrow + g] ? 1.f : 0.f, c0);
                r[1] = make_float4(s0, __builtin_fmaf(a, dt, v), k, __builtin_fmaf(v, dt, a * hdt2));
                r[2] = make_float4(a * hdt2, v > 0.f ? vx0 / v : 0.f, v > 0.f ? vy0 / v : 0.f, 0.f);
            }
            __syncthreads();
            // 2. pair terms of every (step, controlled object): item u = (tb,
            // q, lane of the group); the groups never straddle a wave
            const int items = nb * NC * G;
            for (int u0 = 0; u0 < items; u0 += nthr) {   // block-uniform trip count
                const int u = u0 + tid;
                float gx = 0.f, gy = 0.f, gt = 0.f;
                const int grp = u / G, gl = u - grp * G;
                const int tb = grp / max(NC, 1), qq = grp - tb * NC;
                const int i = u < items ? cidx[qq] : 0;
                const int rb = u < items ? tb * maxN : 0;   // the step's row
                // partners that may have a non-zero term: the margin is at most
                // r_i + r_j - d / sqrt(2) (r <= half length + half width), and
                // below -kCullGap the exponential of the term overflows, so the
                // term is exactly +-0
                uint32_t near = 0;   // bit e: partner gl + e G
                if (u < items) {
                    const float4 pi = tst[rb + i];
                    const float ri = pi.z - kCullGap;   // half length + half width (+- rounding)
                    for (int e = 0, j = gl; j < N; ++e, j += G) {
                        const float4 pj = tst[rb + j];
                        const float dx = pj.x - pi.x, dy = pj.y - pi.y;
                        const float rs = ri + pj.z;
                        // the object itself is never a partner
                        if (j != i && __builtin_fmaf(dy, dy, dx * dx) <= 2.0f * rs * rs)
                            near |= 1u << e;
                    }
                }
                // The wave's marked pairs, lane-major and in ascending partner
                // order within a lane, are evaluated 64 at a time, one per lane;
                // each lane then adds its own terms in that order, so its sums
                // equal those over every partner (adding +-0 changes no sum).
                const int cnt = __popc(near);
                int incl = cnt;
                for (int d = 1; d < 64; d <<= 1) {
                    const int v = __shfl_up(incl, d);
                    if (lane >= d)
                        incl += v;
                }
                const int excl = incl - cnt, total = __shfl(incl, 63);
                uint32_t rem = near;   // marked partners not yet listed
                int listed = 0, added = 0;
                for (int base = 0; base < total; base += 64) {   // wave-uniform
                    while (rem && excl + listed < base + 64) {
                        wslot[excl + listed - base] = (lane << 8) | __builtin_ctz(rem);
                        rem &= rem - 1u;
                        ++listed;
                    }
                    __builtin_amdgcn_wave_barrier();   // the list precedes its reads
                    const bool has = base + lane < total;
                    const int v = wslot[lane];
                    const int src = has ? (v >> 8) & 63 : lane;
                    const int oi = __shfl(i, src), orb = __shfl(rb, src), ogl = __shfl(gl, src);
                    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (has) {
                        const int j = ogl + (v & 31) * G;
                        const float4 pi = st4[orb + oi], pj = st4[orb + j];
                        const float2 hi = st2[orb + oi], hj = st2[orb + j];
                        const Box bi{pi.x, pi.y, pi.z, pi.w, hi.x, hi.y};
                        const Box bj{pj.x, pj.y, pj.z, pj.w, hj.x, hj.y};
                        float ux, uy, ut;
                        // the pair's margin with the lower index first, as in the forward
                        const float m = oi < j ? sat_margin_grad_one(bi, bj, false, ux, uy, ut)
                                               : sat_margin_grad_one(bj, bi, true, ux, uy, ut);
                        // the sigmoid's derivative only scales a gradient term:
                        // the hardware exponential and reciprocal (about 1 ulp)
                        const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-m * (1.0f / kSoftScale)));
                        const float dm = sg * (1.0f - sg) * (1.0f / kSoftScale);
                        // selects, not products: an invalid object's values may be
                        // anything (the bound never marks the object itself)
                        const bool ok = hj.x >= 0.f;
                        r = make_float4(ok ? dm * ux : 0.f, ok ? dm * uy : 0.f, ok ? dm * ut : 0.f, 0.f);
                    }
                    wres[lane] = r;
                    __builtin_amdgcn_wave_barrier();   // the terms precede their reads
                    while (added < cnt && excl + added < base + 64) {
                        const float4 t = wres[excl + added - base];
                        gx += t.x;
                        gy += t.y;
                        gt += t.z;
                        ++added;
                    }
                    __builtin_amdgcn_wave_barrier();   // the reads precede the next batch's writes
                }
                for (int d = G >> 1; d > 0; d >>= 1) {   // fixed tree within the group
                    gx += __shfl_xor(gx, d);
                    gy += __shfl_xor(gy, d);
                    gt += __shfl_xor(gt, d);
                }
                if (u < items && gl == 0) {
                    float *pp = part + 3 * (tb * maxN + qq);
                    pp[0] = gx;
                    pp[1] = gy;
                    pp[2] = gt;
                }
            }
            __syncthreads();
            // 3. reverse recursion over the block's steps, one thread per
            // controlled object
            if (q < NC) {
                const int i = i_own;
                const long g = g_own;
                for (int t = tb_hi; t > tb_lo; --t) {
                    const int tb = t - tb_lo - 1, at = tb * maxN + i;
                    const float *pp = part + 3 * (tb * maxN + q);
                    const float4 *r = (const float4 *)(rec + kBwdRec * (tb * maxN + q));
                    bx += w * pp[0];
                    by += w * pp[1];
                    byaw += w * pp[2];
                    const float4 pa = st4[at], r0 = r[0], r1 = r[1], r2 = r[2];
                    if (r0.z != 0.f) {
                        bx += w * 2.f * (pa.x - r0.x);
                        by += w * 2.f * (pa.y - r0.y);
                    }
                    // factors from the previous state (t - 1) and the action of step t
                    const float c0 = r0.w, s0 = r1.x, nv = r1.y, k = r1.z, dist = r1.w;
                    const float ahdt2 = r2.x, ux = r2.y, uy = r2.z;
                    const float ns = pa.w, nc = pa.z;   // sin, cos of the yaw at t
                    const float bnv = __builtin_fmaf(bvx, nc, bvy * ns);
                    const float tyaw = byaw + nv * __builtin_fmaf(bvy, nc, -(bvx * ns));
                    const float ga_ =
                        __builtin_fmaf(hdt2, __builtin_fmaf(bx, c0, __builtin_fmaf(by, s0, k * tyaw)), dt * bnv);
                    const float gk_ = dist * tyaw;
                    const float pyaw = tyaw + ahdt2 * __builtin_fmaf(by, c0, -(bx * s0));
                    const float bv = __builtin_fmaf(k * dt, tyaw, bnv);
                    A.grad_a[(long)(t - 1) * n + g] = ga_;
                    A.grad_k[(long)(t - 1) * n + g] = gk_;
                    byaw = pyaw;
                    bvx = __builtin_fmaf(dt, bx, bv * ux);
                    bvy = __builtin_fmaf(dt, by, bv * uy);
                }
            }
            __syncthreads();   // the block's LDS is reused by the next block
        }
    }
}

// Steps per LDS block for this object bound and checkpoint interval.
int backward_block_steps(int maxN, int K)
{
    const size_t per_step = (size_t)maxN * kBwdStepBytes;
    int sb = (int)(kBwdStageBudget / (per_step > 0 ? per_step : 1));
    return sb < 1 ? 1 : (sb > K ? K : sb);
}

static size_t backward_lds(int maxN, int SB)
{
    return backward_wave_offset(maxN, SB) + (size_t)kBwdThreads / 64 * 64 * (16 + 4);
}

void launch_backward(const BackwardArgs &a, hipStream_t st)
{
    const size_t lds = backward_lds(a.maxN, a.SB);
    if (lds > 65536)
        // a failure here makes the launch below fail, which the caller reports
        (void)hipFuncSetAttribute((const void *)k_rollout_backward, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_rollout_backward, dim3(a.S), dim3(kBwdThreads), lds, st, a);
}

} // namespace wm
