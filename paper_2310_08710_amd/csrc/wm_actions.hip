// wm_actions.hip -- the delta action space (App. A.1) and discretized actions
// (Sec. 5.2, Expert).  Elementwise, HBM-bound kernels.
#include "wm_device.h"
#include "wm_internal.h"

namespace wm {

// One block per scenario, so that one-scenario views of a batch stay in range.
__global__ __launch_bounds__(256) void k_delta_step(const int32_t *__restrict__ obj_off, wm_state cur,
                                                    wm_delta_action act, wm_state log_next, wm_state next, float dt)
{
    const int s = blockIdx.x;
    for (int g = obj_off[s] + (int)threadIdx.x; g < obj_off[s + 1]; g += blockDim.x) {
        const wm_state &src = act.controlled[g] ? cur : log_next;
        float x = src.x[g], y = src.y[g], yaw = src.yaw[g], vx = src.vx[g], vy = src.vy[g];
        const uint8_t valid = src.valid[g];
        if (act.controlled[g] && valid) {
            const float nx = x + act.dx[g], ny = y + act.dy[g];
            vx = (nx - x) / dt;
            vy = (ny - y) / dt;
            x = nx;
            y = ny;
            yaw = yaw + act.dyaw[g];
        }
        next.x[g] = x;
        next.y[g] = y;
        next.yaw[g] = yaw;
        next.vx[g] = vx;
        next.vy[g] = vy;
        next.length[g] = src.length[g];
        next.width[g] = src.width[g];
        next.valid[g] = valid;
    }
}

__global__ __launch_bounds__(256) void k_delta_inverse(int n, wm_state cur, wm_state nxt, float *__restrict__ dx,
                                                       float *__restrict__ dy, float *__restrict__ dyaw,
                                                       uint8_t *__restrict__ vout)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n)
        return;
    const bool ok = cur.valid[g] && nxt.valid[g];
    dx[g] = ok ? nxt.x[g] - cur.x[g] : 0.f;
    dy[g] = ok ? nxt.y[g] - cur.y[g] : 0.f;
    dyaw[g] = ok ? nxt.yaw[g] - cur.yaw[g] : 0.f;
    if (vout)
        vout[g] = (uint8_t)ok;
}

// scale = fl((bins - 1) / (hi - lo)) and step = fl((hi - lo) / (bins - 1)) are
// computed once on the host (IEEE binary32).
__global__ __launch_bounds__(256) void k_discretize(int n, const float *__restrict__ v, float lo, float scale,
                                                    float step, int bins, int32_t *__restrict__ index,
                                                    float *__restrict__ snapped)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float d = v[i] - lo;
    const float u = d * scale;
    const float w = u + 0.5f;
    int k = (w >= 0.f) ? (int)fminf(floorf(w), (float)(bins - 1)) : 0;
    k = max(0, min(k, bins - 1));
    index[i] = k;
    if (snapped)
        snapped[i] = lo + (float)k * step;
}

void launch_delta_step(const wm_batch &b, const wm_state &cur, const wm_delta_action &act, const wm_state &log_next,
                       const wm_state &next, float dt, hipStream_t st)
{
    hipLaunchKernelGGL(k_delta_step, dim3(b.num_scenarios), dim3(256), 0, st, b.obj_off, cur, act, log_next, next, dt);
}

void launch_delta_inverse(int n, const wm_state &cur, const wm_state &nxt, float *dx, float *dy, float *dyaw,
                          uint8_t *vout, hipStream_t st)
{
    hipLaunchKernelGGL(k_delta_inverse, dim3((n + 255) / 256), dim3(256), 0, st, n, cur, nxt, dx, dy, dyaw, vout);
}

void launch_discretize(int n, const float *v, float lo, float scale, float step, int bins, int32_t *index,
                       float *snapped, hipStream_t st)
{
    hipLaunchKernelGGL(k_discretize, dim3((n + 255) / 256), dim3(256), 0, st, n, v, lo, scale, step, bins, index,
                       snapped);
}

} // namespace wm
