// wm_backward.hip -- hand-written adjoint of the fused rollout's training
// loss with respect to the actions (differentiable simulation, Sec. 1 and
// Sec. 6; dynamics of App. A.1).
//
// One work-group per scenario.  The forward pass stored the state every K
// steps; each segment [cK, min(cK + K, T)] is recomputed from its checkpoint
// with the same device code as the forward (bit-identical states), written to
// the workspace, and swept in reverse:
//   1. loss adjoint at step t: 2 (p - p_log) for controlled objects, plus
//      sigmoid'(m / 0.1) / 0.1 * dm/d(x, y, yaw) for every pair with a
//      controlled member (each controlled object gathers its own side of
//      every pair, split over threads and summed in a fixed order);
//   2. back through the bicycle step t: gradients of (a, kappa) at t-1 and
//      the adjoint of the previous state.
// Only controlled, valid objects carry adjoints: replayed objects do not
// depend on the actions and frozen objects never enter the loss.
#include "wm_device.h"
#include "wm_internal.h"

namespace wm {

constexpr int kBwdThreads = 256;

__global__ __launch_bounds__(kBwdThreads) void k_rollout_backward(BackwardArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int maxN = A.maxN;
    ObjLds L;
    float *f = (float *)smem;
    L.x = f;
    L.y = f + maxN;
    L.yaw = f + 2 * maxN;
    L.vx = f + 3 * maxN;
    L.vy = f + 4 * maxN;
    L.len = f + 5 * maxN;
    L.wid = f + 6 * maxN;
    L.c = f + 7 * maxN;
    L.s = f + 8 * maxN;
    const int PS = maxN > kBwdThreads ? maxN : kBwdThreads;
    float *adj = f + 9 * maxN;                   // [5][maxN] adjoints (x, y, yaw, vx, vy)
    float *part = adj + 5 * maxN;                // [3][PS] pair partials
    int *cidx = (int *)(part + 3 * PS);          // controlled & valid objects
    uint8_t *b8 = (uint8_t *)(cidx + maxN);
    L.valid = b8;
    L.ctrl = b8 + maxN;
    __shared__ int s_nc;

    const int tid = threadIdx.x;
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
    for (int i = tid; i < N; i += kBwdThreads) {
        L.ctrl[i] = A.act.controlled[o0 + i];
        for (int c = 0; c < 5; ++c)
            adj[c * maxN + i] = 0.f;
        const bool live = A.act.controlled[o0 + i] && A.init.valid[o0 + i];
        if (!live)
            for (int t = 0; t < A.T; ++t) {
                A.grad_a[(long)t * n + o0 + i] = 0.f;
                A.grad_k[(long)t * n + o0 + i] = 0.f;
            }
    }
    __syncthreads();
    const int NC = s_nc;
    const int P = NC > 0 ? max(1, kBwdThreads / NC) : 1;
    const int nseg = (A.T + A.K - 1) / A.K;
    float *seg = A.seg;

    for (int c = nseg - 1; c >= 0; --c) {
        const int t0 = c * A.K, t1 = min(A.T, t0 + A.K);
        // recompute the controlled objects' states t0..t1 into the workspace
        for (int q = tid; q < NC; q += kBwdThreads) {
            const long g = o0 + cidx[q];
            float x = A.ckpt.x[(long)c * n + g], y = A.ckpt.y[(long)c * n + g], yaw = A.ckpt.yaw[(long)c * n + g];
            float vx = A.ckpt.vx[(long)c * n + g], vy = A.ckpt.vy[(long)c * n + g];
            for (int t = t0; t <= t1; ++t) {
                if (t > t0)
                    bicycle_forward(x, y, yaw, vx, vy, A.act.accel[(long)(t - 1) * n + g],
                                    A.act.curvature[(long)(t - 1) * n + g], dt);
                float *row = seg + (long)(t - t0) * 5 * n;
                row[g] = x;
                row[n + g] = y;
                row[2 * n + g] = yaw;
                row[3 * n + g] = vx;
                row[4 * n + g] = vy;
            }
        }
        __syncthreads();
        for (int t = t1; t > t0; --t) {
            const float *row = seg + (long)(t - t0) * 5 * n;
            const long lrow = (long)t * n;
            // state at t: controlled from the recomputation, others from the log
            for (int i = tid; i < N; i += kBwdThreads) {
                const long g = o0 + i;
                float x, y, yaw, len, wid;
                uint8_t v;
                if (L.ctrl[i]) {
                    v = A.init.valid[g];
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
                L.x[i] = x;
                L.y[i] = y;
                L.yaw[i] = yaw;
                L.len[i] = len;
                L.wid[i] = wid;
                L.valid[i] = v;
                float sn, cs;
                sincosf(yaw, &sn, &cs);
                L.c[i] = cs;
                L.s[i] = sn;
            }
            __syncthreads();
            // pair partials: work item (q = controlled slot, p = partner split)
            for (int wi = tid; wi < NC * P; wi += kBwdThreads) {
                const int q = wi % NC, p = wi / NC;
                const int i = cidx[q];
                float gx = 0.f, gy = 0.f, gt = 0.f;
                Box bi;
                bi.x = L.x[i]; bi.y = L.y[i]; bi.c = L.c[i]; bi.s = L.s[i];
                bi.hl = 0.5f * L.len[i]; bi.hw = 0.5f * L.wid[i];
                for (int j = p; j < N; j += P) {
                    if (j == i || !L.valid[j])
                        continue;
                    Box bj;
                    bj.x = L.x[j]; bj.y = L.y[j]; bj.c = L.c[j]; bj.s = L.s[j];
                    bj.hl = 0.5f * L.len[j]; bj.hw = 0.5f * L.wid[j];
                    float ga[3], gb[3], m;
                    if (i < j) {
                        m = sat_margin(bi, bj);
                        sat_margin_grad(bi, bj, ga, gb);
                    } else {
                        m = sat_margin(bj, bi);
                        sat_margin_grad(bj, bi, gb, ga);
                    }
                    const float sg = 1.0f / (1.0f + expf(-m * (1.0f / kSoftScale)));
                    const float dm = sg * (1.0f - sg) * (1.0f / kSoftScale);
                    gx = __builtin_fmaf(dm, ga[0], gx);
                    gy = __builtin_fmaf(dm, ga[1], gy);
                    gt = __builtin_fmaf(dm, ga[2], gt);
                }
                part[wi] = gx;
                part[PS + wi] = gy;
                part[2 * PS + wi] = gt;
            }
            __syncthreads();
            // per controlled object: add the loss adjoint, then step back through t
            for (int q = tid; q < NC; q += kBwdThreads) {
                const int i = cidx[q];
                const long g = o0 + i;
                float px = 0.f, py = 0.f, pt = 0.f;
                for (int p = 0; p < P; ++p) {
                    px += part[p * NC + q];
                    py += part[PS + p * NC + q];
                    pt += part[2 * PS + p * NC + q];
                }
                float bx = adj[i] + w * px, by = adj[maxN + i] + w * py, byaw = adj[2 * maxN + i] + w * pt;
                const float bvx = adj[3 * maxN + i], bvy = adj[4 * maxN + i];
                if (A.log.valid[lrow + g]) {
                    bx += w * 2.f * (L.x[i] - A.log.x[lrow + g]);
                    by += w * 2.f * (L.y[i] - A.log.y[lrow + g]);
                }
                // previous state (t - 1) and the action of step t
                const float *prow = seg + (long)(t - 1 - t0) * 5 * n;
                const float yaw0 = prow[2 * n + g], vx0 = prow[3 * n + g], vy0 = prow[4 * n + g];
                const float a = A.act.accel[(long)(t - 1) * n + g], k = A.act.curvature[(long)(t - 1) * n + g];
                const float v = sqrtf(__builtin_fmaf(vy0, vy0, vx0 * vx0));
                const float dist = __builtin_fmaf(v, dt, a * hdt2);
                const float nv = __builtin_fmaf(a, dt, v);
                const float nyaw = L.yaw[i];
                float ns, nc;
                sincosf(nyaw, &ns, &nc);
                float s0, c0;
                sincosf(yaw0, &s0, &c0);
                const float bnv = __builtin_fmaf(bvx, nc, bvy * ns);
                const float tyaw = byaw + nv * __builtin_fmaf(bvy, nc, -(bvx * ns));
                const float ga_ = __builtin_fmaf(hdt2, __builtin_fmaf(bx, c0, __builtin_fmaf(by, s0, k * tyaw)), dt * bnv);
                const float gk_ = dist * tyaw;
                const float pyaw = tyaw + a * hdt2 * __builtin_fmaf(by, c0, -(bx * s0));
                const float bv = __builtin_fmaf(k * dt, tyaw, bnv);
                const float inv = v > 0.f ? bv / v : 0.f;
                A.grad_a[(long)(t - 1) * n + g] = ga_;
                A.grad_k[(long)(t - 1) * n + g] = gk_;
                adj[i] = bx;
                adj[maxN + i] = by;
                adj[2 * maxN + i] = pyaw;
                adj[3 * maxN + i] = __builtin_fmaf(dt, bx, inv * vx0);
                adj[4 * maxN + i] = __builtin_fmaf(dt, by, inv * vy0);
            }
            __syncthreads();
        }
    }
}

static size_t backward_lds(int maxN)
{
    const size_t ps = maxN > kBwdThreads ? (size_t)maxN : (size_t)kBwdThreads;
    return align_up((size_t)maxN * (9 + 5) * 4 + 3 * ps * 4 + (size_t)maxN * 4 + 2 * (size_t)maxN, 16);
}

void launch_backward(const BackwardArgs &a, hipStream_t st)
{
    const size_t lds = backward_lds(a.maxN);
    if (lds > 65536)
        // a failure here makes the launch below fail, which the caller reports
        (void)hipFuncSetAttribute((const void *)k_rollout_backward, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_rollout_backward, dim3(a.S), dim3(kBwdThreads), lds, st, a);
}

} // namespace wm
