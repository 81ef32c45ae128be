// wm_backward.hip -- hand-written adjoint of the fused rollout's training
// loss with respect to the actions (differentiable simulation, Sec. 1 and
// Sec. 6; dynamics of App. A.1).
//
// The reverse sweep's only sequential part is the recursion of each
// controlled object's adjoint through the bicycle steps; everything it
// consumes is independent of the adjoint.  So the adjoint runs as three
// launches:
//   A. k_bwd_recompute, one work-group per (scenario, checkpoint segment),
//      one thread per controlled object: the forward stored the state
//      every K steps; each segment is recomputed from its checkpoint with the
//      forward's own device code (bit-identical states), and for every step
//      t the recursion's inputs are written to the workspace: the state at t
//      (position, cosine and sine of the yaw), the log at t, and the factors
//      of the step's derivatives that the state at t - 1 and the action give
//      (sine and cosine of the previous yaw, speeds, distance, velocity
//      direction).  Segments are independent, so all of them run at once.
//   B. k_bwd_pairs, one work-group per (scenario, block of SB steps): the
//      loss gradient with respect to each controlled object's (x, y, yaw) at
//      each step, sigmoid'(m / 0.1) / 0.1 * dm/d(x, y, yaw) over every pair
//      with a controlled member.  A group of G lanes per (step, controlled
//      object) splits the partners (j = lane, lane + G, ...) and sums with a
//      fixed shuffle tree.  A lane first marks the partners close enough for
//      a non-zero term (a distance bound); the wave evaluates its marked pairs
//      one per lane, and each lane adds its own terms in ascending partner
//      order.  It also writes the zero gradients of the block's steps for
//      the objects that are not differentiated.
//   C. k_bwd_reverse, one work-group per scenario, one thread per
//      controlled object: the reverse recursion over all T steps, the
//      log-divergence term 2 (p - p_log) and the pair terms added, then back
//      through the bicycle step, with the adjoint in registers and each
//      step's inputs loaded several steps ahead.
// G depends only on the scenario's object count, so the gradients are
// identical for every checkpoint interval and every blocking.  Only
// controlled, valid objects carry adjoints: replayed objects do not depend on
// the actions and frozen objects never enter the loss.
#include "wm_device.h"
#include "wm_internal.h"

namespace wm {

// Pair terms whose margin is below -kCullGap are skipped: there -m / kSoftScale
// exceeds 128 / log2(e), the FP32 exponential of the sigmoid overflows to
// infinity and the term is exactly zero.
constexpr float kCullGap = 9.0f;
static_assert(kCullGap / kSoftScale * 1.4426950f > 129.0f, "skipped terms overflow the exponential");
static_assert(WM_MAX_OBJECTS <= 64 * 32, "a lane's partners fit in one 32-bit mask");

constexpr int kRecThreads = 64;
constexpr int kRecBatch = 8;     // recomputed steps whose inputs are loaded together
constexpr int kPairThreads = 512;
constexpr int kRevThreads = 256;
constexpr size_t kPairStepBytes = 16 + 8;        // LDS per step and object in k_bwd_pairs
constexpr size_t kPairStageBudget = 24 * 1024;
constexpr int kPairMaxSteps = 16;
constexpr int kPairBatch = 4;    // staged (step, object) items per thread with loads in flight together


// The recursion's inputs of step t = 1..T and object g: four float4 at
// rec + 4 ((t - 1) n + g):
//   [0] state at t: x, y, cos and sin of the yaw
//   [1] log at t: x, y, valid (1 or 0); cos of the yaw at t - 1
//   [2] sin of the yaw at t - 1; v + a dt; curvature; v dt + a dt^2 / 2
//   [3] a dt^2 / 2; velocity direction at t - 1 (0, 0 at v = 0); 0
// and the pair-term sums (x, y, yaw, 0) at part + ((t - 1) n + g).
static_assert(kRecFields == 16, "four float4 per step and object");

// The controlled, valid objects of scenario s (scenario-local indices, in
// index order) into cidx; returns their count.  Work-group-wide (blockDim a
// multiple of 64, wcnt holds blockDim / 64 entries); ends with a barrier.
// With `kind`, also each object's kind: 2 controlled and valid, 1
// controlled and invalid, 0 replayed from the log.
__device__ __forceinline__ int live_objects(const BackwardArgs &A, int o0, int N, int *cidx, int *wcnt,
                                            uint8_t *kind = nullptr)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int run = 0;
    for (int i0 = 0; i0 < N; i0 += blockDim.x) {   // block-uniform
        const int i = i0 + threadIdx.x;
        const bool ctl = i < N && A.act.controlled[o0 + i];
        const bool live = ctl && A.init.valid[o0 + i];
        if (kind && i < N)
            kind[i] = ctl ? (live ? 2 : 1) : 0;
        const uint64_t bal = __ballot(live);
        if (lane == 0)
            wcnt[wv] = __popcll(bal);
        __syncthreads();
        int before = 0, tot = 0;
        for (int v = 0; v < nw; ++v) {
            before += v < wv ? wcnt[v] : 0;
            tot += wcnt[v];
        }
        if (live)
            cidx[run + before + __popcll(bal & ((1ull << lane) - 1ull))] = i;
        run += tot;
        __syncthreads();
    }
    return run;
}

// A. ------------------------------------------------------------------------
// One work-group per (scenario, checkpoint segment), one thread per
// controlled object: the segment is recomputed from its checkpoint.
__global__ __launch_bounds__(kRecThreads) void k_bwd_recompute(BackwardArgs A)
{
    __shared__ int cidx[WM_MAX_OBJECTS];
    __shared__ int wcnt[kRecThreads / 64];
    const int nseg = (A.T + A.K - 1) / A.K;
    const int s = blockIdx.x / nseg, c = blockIdx.x - s * nseg;
    const int t0 = c * A.K, t1 = min(A.T, t0 + A.K);
    const int o0 = A.obj_off[s], N = A.obj_off[s + 1] - o0;
    const long n = A.n;
    const int NC = live_objects(A, o0, N, cidx, wcnt);
    const float dt = A.dt, hdt2 = 0.5f * dt * dt;
    for (int q = threadIdx.x; q < NC; q += kRecThreads) {
        const long g = o0 + cidx[q];
        float x = A.ckpt.x[(long)c * n + g], y = A.ckpt.y[(long)c * n + g], yaw = A.ckpt.yaw[(long)c * n + g];
        float vx = A.ckpt.vx[(long)c * n + g], vy = A.ckpt.vy[(long)c * n + g];
        for (int tb = t0; tb < t1; tb += kRecBatch) {
          // the batch's actions and logs, every load in flight together
          float ba[kRecBatch], bk[kRecBatch], blx[kRecBatch], bly[kRecBatch];
          uint8_t blv[kRecBatch];
#pragma unroll
          for (int u = 0; u < kRecBatch; ++u) {
              const int t = min(tb + u, t1 - 1);
              ba[u] = A.act.accel[(long)t * n + g];
              bk[u] = A.act.curvature[(long)t * n + g];
              blx[u] = A.log.x[(long)(t + 1) * n + g];
              bly[u] = A.log.y[(long)(t + 1) * n + g];
              blv[u] = A.log.valid[(long)(t + 1) * n + g];
          }
#pragma unroll
          for (int u = 0; u < kRecBatch; ++u) {
            const int t = tb + u;   // step t + 1 from the state at t
            if (t >= t1)
                break;
            const float a = ba[u], k = bk[u];
            const float v = sqrtf(__builtin_fmaf(vy, vy, vx * vx));
            const float ux = v > 0.f ? vx / v : 0.f, uy = v > 0.f ? vy / v : 0.f;
            float s0, c0, sn, cs;
            bicycle_forward_sc(x, y, yaw, vx, vy, a, k, dt, s0, c0, sn, cs);
            float4 *r = (float4 *)A.rec + 4 * ((long)t * n + g);
            r[0] = make_float4(x, y, cs, sn);
            r[1] = make_float4(blx[u], bly[u], blv[u] ? 1.f : 0.f, c0);
            r[2] = make_float4(s0, __builtin_fmaf(a, dt, v), k, __builtin_fmaf(v, dt, a * hdt2));
            r[3] = make_float4(a * hdt2, ux, uy, 0.f);
          }
        }
    }
}

// B. ------------------------------------------------------------------------
// Byte offset of the per-wave pair lists in k_bwd_pairs' LDS: after the step
// blocks, the controlled indices and the object kinds.
__host__ __device__ constexpr size_t pair_wave_offset(int maxN, int SB)
{
    return ((size_t)SB * maxN * kPairStepBytes + (size_t)maxN * 5 + 15) / 16 * 16;
}

__global__ __launch_bounds__(kPairThreads) void k_bwd_pairs(BackwardArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int maxN = A.maxN, SB = A.SB;
    const int nblk = (A.T + SB - 1) / SB;
    const int s = blockIdx.x / nblk, blk = blockIdx.x - s * nblk;
    const int tb_lo = blk * SB, nb = min(A.T, tb_lo + SB) - tb_lo;   // steps tb_lo + 1 .. tb_lo + nb
    // LDS: [SB][maxN] (x, y, cos, sin), [SB][maxN] (half length or -1 when
    // invalid, half width); the controlled objects' indices; per object 2
    // (controlled and valid), 1 (controlled, invalid) or 0 (from the log)
    float4 *st4 = (float4 *)smem;
    float2 *st2 = (float2 *)(st4 + SB * maxN);
    int *cidx = (int *)(st2 + SB * maxN);
    uint8_t *kind = (uint8_t *)(cidx + maxN);
    // per wave: the list of marked pairs being evaluated and their terms
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float4 *wres = (float4 *)(smem + pair_wave_offset(maxN, SB)) + 64 * wv;
    int *wslot = (int *)(smem + pair_wave_offset(maxN, SB) + (size_t)kPairThreads / 64 * 64 * 16) + 64 * wv;
    __shared__ int wcnt[kPairThreads / 64];

    const int tid = threadIdx.x, nthr = blockDim.x;
    const int o0 = A.obj_off[s], N = A.obj_off[s + 1] - o0;
    const long n = A.n;

    // each object's kind; the controlled, valid objects in index order
    const int NC = live_objects(A, o0, N, cidx, wcnt, kind);
    // the objects that are not differentiated get zero gradients at the
    // block's steps (actions tb_lo .. tb_lo + nb - 1)
    for (int it = tid; it < nb * N; it += nthr) {
        const int tb = it / N, i = it - tb * N;
        if (kind[i] != 2) {
            const long at = (long)(tb_lo + tb) * n + o0 + i;
            A.grad_a[at] = 0.f;
            A.grad_k[at] = 0.f;
        }
    }
    if (NC == 0)
        return;   // work-group uniform
    // partner split: G lanes (a power of two <= 64) per (step, controlled
    // object), about 16 partners each
    int G = 1;
    while (G < 64 && G * 16 < N)
        G <<= 1;

    // 1. states of every object at the block's steps (slot tb = t - tb_lo - 1),
    // kPairBatch items per thread with their loads in flight together
    for (int it0 = tid; it0 < nb * N; it0 += nthr * kPairBatch) {
        float x[kPairBatch], y[kPairBatch], yw[kPairBatch], cs[kPairBatch], len[kPairBatch], wid[kPairBatch];
        uint8_t vv[kPairBatch], kd[kPairBatch];
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u) {
            const int it = min(it0 + nthr * u, nb * N - 1);
            const int tb = it / N, i = it - tb * N;
            const int t = tb_lo + 1 + tb;
            const long g = o0 + i, lrow = (long)t * n;
            kd[u] = kind[i];
            if (kd[u] == 2) {
                const float4 r = ((const float4 *)A.rec)[4 * ((long)(t - 1) * n + g)];
                x[u] = r.x;
                y[u] = r.y;
                cs[u] = r.z;
                yw[u] = r.w;   // the sine
                vv[u] = 1;
                len[u] = A.init.length[g];
                wid[u] = A.init.width[g];
            } else if (kd[u] == 1) {   // controlled and invalid: frozen, never a partner
                x[u] = A.init.x[g];
                y[u] = A.init.y[g];
                yw[u] = A.init.yaw[g];
                vv[u] = 0;
                len[u] = A.init.length[g];
                wid[u] = A.init.width[g];
            } else {
                x[u] = A.log.x[lrow + g];
                y[u] = A.log.y[lrow + g];
                yw[u] = A.log.yaw[lrow + g];
                vv[u] = A.log.valid[lrow + g];
                len[u] = A.log.length[lrow + g];
                wid[u] = A.log.width[lrow + g];
            }
        }
#pragma unroll
        for (int u = 0; u < kPairBatch; ++u) {
            const int it = it0 + nthr * u;
            if (it >= nb * N)
                break;
            const int tb = it / N, i = it - tb * N;
            float sn, c;
            if (kd[u] == 2) {
                c = cs[u];
                sn = yw[u];
            } else {
                sincosf(yw[u], &sn, &c);
            }
            const int at = tb * maxN + i;
            const float hl = vv[u] ? 0.5f * len[u] : -1.f, hw = 0.5f * wid[u];
            st4[at] = make_float4(x[u], y[u], c, sn);
            st2[at] = make_float2(hl, hw);
        }
    }
    __syncthreads();

    // 2. pair terms of every (step, controlled object): item u = (tb, q,
    // lane of the group); the groups never straddle a wave
    const int items = nb * NC * G;
    for (int u0 = 0; u0 < items; u0 += nthr) {   // block-uniform trip count
        const int u = u0 + tid;
        float gx = 0.f, gy = 0.f, gt = 0.f;
        const int grp = u / G, gl = u - grp * G;
        const int tb = grp / NC, qq = grp - tb * NC;
        const int i = u < items ? cidx[qq] : 0;
        const int rb = u < items ? tb * maxN : 0;   // the step's row
        // partners that may have a non-zero term: the margin is at most
        // r_i + r_j - d / sqrt(2) (r <= half length + half width), and below
        // -kCullGap the exponential of the term overflows, so the term is
        // exactly +-0
        uint32_t near = 0;   // bit e: partner gl + e G
        if (u < items) {
            const float4 pi = st4[rb + i];
            const float2 hi = st2[rb + i];
            const float ri = hi.x + hi.y + kCullGap;   // half length + half width + the gap
            for (int e = 0, j = gl; j < N; ++e, j += G) {
                const float4 pj = st4[rb + j];
                const float2 hj = st2[rb + j];
                const float dx = pj.x - pi.x, dy = pj.y - pi.y;
                const float rs = ri + (hj.x + hj.y);   // an invalid partner's reach is 1 m short: never needed
                // the object itself is never a partner
                if (j != i && __builtin_fmaf(dy, dy, dx * dx) <= 2.0f * rs * rs)
                    near |= 1u << e;
            }
        }
        // The wave's marked pairs, lane-major and in ascending partner order
        // within a lane, are evaluated 64 at a time, one per lane; each lane
        // then adds its own terms in that order, so its sums equal those over
        // every partner (adding +-0 changes no sum).
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
                // the sigmoid's derivative only scales a gradient term: the
                // hardware exponential and reciprocal (about 1 ulp)
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
            const int t = tb_lo + 1 + tb;
            ((float4 *)A.part)[(long)(t - 1) * n + o0 + i] = make_float4(gx, gy, gt, 0.f);
        }
    }
}

// C. ------------------------------------------------------------------------
// One work-group per scenario, one thread per controlled object.  A thread's
// inputs for a step come from the workspace (coalesced over the scenario's
// objects) kRevDepth steps ahead of their use, in a ring of registers, so
// the recursion's chain does not wait for memory.
constexpr int kRevDepth = 8;

struct RevStep {
    float4 p, r0, r1, r2, r3;   // pair sums; the recursion's inputs (layout above)
};

__device__ __forceinline__ RevStep rev_load(const BackwardArgs &A, int t, long g)
{
    const long at = (long)(t - 1) * A.n + g;
    const float4 *r = (const float4 *)A.rec + 4 * at;
    return RevStep{((const float4 *)A.part)[at], r[0], r[1], r[2], r[3]};
}

// One step of the reverse recursion for one controlled object: the log and
// pair terms of step t, then the bicycle adjoint back to step t - 1.
__device__ __forceinline__ void rev_step(const BackwardArgs &A, const RevStep &cur, int t, long g, float w,
                                         float &bx, float &by, float &byaw, float &bvx, float &bvy)
{
    const float dt = A.dt, hdt2 = 0.5f * dt * dt;
    const long n = A.n;
    bx += w * cur.p.x;
    by += w * cur.p.y;
    byaw += w * cur.p.z;
    if (cur.r1.z != 0.f) {   // log term, where the log is valid
        bx += w * 2.f * (cur.r0.x - cur.r1.x);
        by += w * 2.f * (cur.r0.y - cur.r1.y);
    }
    // factors from the previous state (t - 1) and the action of step t
    const float nc = cur.r0.z, ns = cur.r0.w, c0 = cur.r1.w, s0 = cur.r2.x;
    const float nv = cur.r2.y, k = cur.r2.z, dist = cur.r2.w;
    const float ahdt2 = cur.r3.x, ux = cur.r3.y, uy = cur.r3.z;
    const float bnv = __builtin_fmaf(bvx, nc, bvy * ns);
    const float tyaw = byaw + nv * __builtin_fmaf(bvy, nc, -(bvx * ns));
    const float ga_ = __builtin_fmaf(hdt2, __builtin_fmaf(bx, c0, __builtin_fmaf(by, s0, k * tyaw)), dt * bnv);
    const float gk_ = dist * tyaw;
    const float pyaw = tyaw + ahdt2 * __builtin_fmaf(by, c0, -(bx * s0));
    const float bv = __builtin_fmaf(k * dt, tyaw, bnv);
    A.grad_a[(long)(t - 1) * n + g] = ga_;
    A.grad_k[(long)(t - 1) * n + g] = gk_;
    byaw = pyaw;
    bvx = __builtin_fmaf(dt, bx, bv * ux);
    bvy = __builtin_fmaf(dt, by, bv * uy);
}

// Scenarios with at most 64 controlled objects (one wave of the recursion):
// the other waves stage the inputs of a chunk of steps in LDS, two buffers
// of kRevStage bytes, while the first wave runs the recursion over the
// previous chunk from LDS.
constexpr int kRevStage = 24576;
constexpr int kRevF4 = 5;   // float4 per (step, object): pair sums + 4 of the record
constexpr int kRevBatch = 8;

__global__ __launch_bounds__(kRevThreads) void k_bwd_reverse(BackwardArgs A)
{
    __shared__ int cidx[WM_MAX_OBJECTS];
    __shared__ int wcnt[kRevThreads / 64];
    extern __shared__ __align__(16) float4 rstage[];
    const int s = blockIdx.x;
    const int o0 = A.obj_off[s], N = A.obj_off[s + 1] - o0;
    const int NC = live_objects(A, o0, N, cidx, wcnt);
    const float w = A.dloss[s];
    const int T = A.T;
    if (NC == 0)
        return;
    if (NC <= 64 && kRevThreads >= 128) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int C = max(1, min(T, kRevStage / (16 * kRevF4 * NC)));   // steps per chunk
        const int nchunk = (T + C - 1) / C;
        const long n = A.n;
        // chunk c holds steps t = T - c C down to max(1, T - (c + 1) C + 1):
        // element (u, q, r) at ((u * NC + q) * kRevF4 + r) of its buffer
        // (kRevBatch loads of a thread in flight together)
        auto stage_chunk = [&](int c, int first, int stride) {
            float4 *buf = rstage + (long)(c & 1) * (kRevStage / 16);
            const int thi = T - c * C, nstep = min(C, thi);
            const int items = nstep * NC * kRevF4;
            for (int e0 = first; e0 < items; e0 += kRevBatch * stride) {
                float4 v[kRevBatch];
#pragma unroll
                for (int b = 0; b < kRevBatch; ++b) {
                    const int e = min(e0 + b * stride, items - 1);
                    const int r = e % kRevF4, uq = e / kRevF4, q = uq % NC, u = uq / NC;
                    const long at = (long)(thi - u - 1) * n + o0 + cidx[q];
                    v[b] = r == 0 ? ((const float4 *)A.part)[at] : ((const float4 *)A.rec)[4 * at + (r - 1)];
                }
#pragma unroll
                for (int b = 0; b < kRevBatch; ++b)
                    if (e0 + b * stride < items)
                        buf[e0 + b * stride] = v[b];
            }
        };
        stage_chunk(0, threadIdx.x, kRevThreads);
        __syncthreads();
        float bx = 0.f, by = 0.f, byaw = 0.f, bvx = 0.f, bvy = 0.f;
        const long g = lane < NC ? o0 + cidx[lane] : 0;
        for (int c = 0; c < nchunk; ++c) {
            if (wv > 0) {
                if (c + 1 < nchunk)
                    stage_chunk(c + 1, threadIdx.x - 64, kRevThreads - 64);
            } else if (lane < NC) {
                const float4 *buf = rstage + (long)(c & 1) * (kRevStage / 16);
                const int thi = T - c * C, nstep = min(C, thi);
                for (int u = 0; u < nstep; ++u) {
                    const float4 *e = buf + (u * NC + lane) * kRevF4;
                    const RevStep cur{e[0], e[1], e[2], e[3], e[4]};
                    rev_step(A, cur, thi - u, g, w, bx, by, byaw, bvx, bvy);
                }
            }
            __syncthreads();
        }
        return;
    }
    for (int q = threadIdx.x; q < NC; q += kRevThreads) {
        const long g = o0 + cidx[q];
        // the adjoint of the object's (x, y, yaw, vx, vy)
        float bx = 0.f, by = 0.f, byaw = 0.f, bvx = 0.f, bvy = 0.f;
        RevStep ring[kRevDepth];
#pragma unroll
        for (int u = 0; u < kRevDepth; ++u)
            ring[u] = rev_load(A, max(T - u, 1), g);
        for (int t0 = T; t0 >= 1; t0 -= kRevDepth) {
#pragma unroll
            for (int u = 0; u < kRevDepth; ++u) {
                const int t = t0 - u;
                if (t < 1)
                    break;
                const RevStep cur = ring[u];
                if (t - kRevDepth >= 1)   // in flight while the next steps run
                    ring[u] = rev_load(A, t - kRevDepth, g);
                rev_step(A, cur, t, g, w, bx, by, byaw, bvx, bvy);
            }
        }
    }
}

// Steps per pair work-group for this object bound.
int backward_block_steps(int maxN, int K)
{
    (void)K;   // the blocking no longer follows the checkpoint interval
    const size_t per_step = (size_t)(maxN > 0 ? maxN : 1) * kPairStepBytes;
    int sb = (int)(kPairStageBudget / per_step);
    return sb < 1 ? 1 : (sb > kPairMaxSteps ? kPairMaxSteps : sb);
}

static size_t pair_lds(int maxN, int SB)
{
    return pair_wave_offset(maxN, SB) + (size_t)kPairThreads / 64 * 64 * (16 + 4);
}

void launch_backward(const BackwardArgs &a, hipStream_t st)
{
    const int nseg = (a.T + a.K - 1) / a.K;
    hipLaunchKernelGGL(k_bwd_recompute, dim3((unsigned)((long)a.S * nseg)), dim3(kRecThreads), 0, st, a);
    const size_t lds = pair_lds(a.maxN, a.SB);
    if (lds > 65536)
        // a failure here makes the launch below fail, which the caller reports
        (void)hipFuncSetAttribute((const void *)k_bwd_pairs, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int nblk = (a.T + a.SB - 1) / a.SB;
    hipLaunchKernelGGL(k_bwd_pairs, dim3((unsigned)((long)a.S * nblk)), dim3(kPairThreads), lds, st, a);
    hipLaunchKernelGGL(k_bwd_reverse, dim3(a.S), dim3(kRevThreads), 2 * kRevStage, st, a);
}

} // namespace wm
