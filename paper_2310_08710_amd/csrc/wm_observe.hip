// wm_observe.hip -- default observation (Sec. 3.2): objects in the ego frame
// and the k road points nearest to the ego, exact, ascending by
// (binary32 squared distance, index).
//
// One 1024-thread work-group per (scenario, ego) and state row.  Each thread keeps up to 32
// keys in registers (points j = tid + 1024 r), so a scenario's road graph is
// read once per ego.  The k-th smallest key is found by a 3-pass radix select
// (11 + 11 + 10 bits of the float bits, which order like the values because
// the keys are non-negative) with LDS histograms; the points with a smaller
// key plus the lowest-index points equal to it are compacted and sorted by a
// bitonic network on (key << 32 | index).
#include "wm_device.h"
#include "wm_internal.h"

namespace wm {

constexpr int kObsThreads = 1024;
constexpr int kObsKeys = WM_MAX_OBSERVE_POINTS / kObsThreads;  // 32
constexpr uint32_t kNoKey = 0xffffffffu;                        // invalid point / padding
constexpr int kHistBins = 2048;                                 // widest radix digit: 11 bits
constexpr int kHistCopies = 4;

__device__ __forceinline__ uint32_t topk_key(float qx, float qy, float ex, float ey)
{
    const float dx = qx - ex, dy = qy - ey;
    const float xx = dx * dx, yy = dy * dy;  // no contraction: fl(fl(dx*dx) + fl(dy*dy))
    return __float_as_uint(xx + yy);
}

// Block-wide exclusive prefix of a per-thread count (wave ballot-free: small
// values); returns the exclusive prefix and writes the block total to *total.
__device__ __forceinline__ int block_exclusive(int v, int *wtot, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(incl, d);
        if (lane >= d)
            incl += u;
    }
    if (lane == 63)
        wtot[w] = incl;
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < kObsThreads / 64; ++i) {
        off += (i < w) ? wtot[i] : 0;
        tot += wtot[i];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

__global__ __launch_bounds__(kObsThreads) void k_observe(ObserveArgs A0)
{
    // grid y: the state row (time step) observed, with its own outputs
    ObserveArgs A = A0;
    if (blockIdx.y > 0) {
        const long t = blockIdx.y, so = t * A0.n, slots = A0.S * A0.E;
        A.st.x += so;
        A.st.y += so;
        A.st.yaw += so;
        A.st.vx += so;
        A.st.vy += so;
        A.st.length += so;
        A.st.width += so;
        A.st.valid += so;
        A.rg_idx += t * slots * A0.k;
        if (A.rg_feat)
            A.rg_feat += t * slots * A0.k * 4;
        if (A.obj_feat)
            A.obj_feat += t * slots * A0.maxN * 8;
    }
    // four copies of the radix histogram, lane l counting into copy l % 4,
    // so that lanes of one wave with equal digits do not all hit one address
    __shared__ int hist[kHistCopies * kHistBins];
    __shared__ int wtot[kObsThreads / 64];
    __shared__ uint64_t sel[1024];
    __shared__ int sh_bin, sh_before, sh_count;
    const int tid = threadIdx.x;
    const int slot = blockIdx.x;                 // s * E + e
    const int s = slot / A.E;
    const int o0 = A.obj_off[s], N = A.obj_off[s + 1] - o0;
    const int p0 = A.rg_off[s], P = A.rg_off[s + 1] - p0;
    const int g = A.ego[slot];
    const long out0 = (long)slot * A.k;
    const bool ego_valid = A.st.valid[g];
    const float ex = A.st.x[g], ey = A.st.y[g];
    float es, ec;
    sincosf(A.st.yaw[g], &es, &ec);

    // ---- objects in the ego frame ----
    if (A.obj_feat) {
        float *of = A.obj_feat + (long)slot * A.maxN * 8;
        for (int j = tid; j < A.maxN; j += kObsThreads) {
            float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (ego_valid && j < N && A.st.valid[o0 + j]) {
                const int h = o0 + j;
                const float dx = A.st.x[h] - ex, dy = A.st.y[h] - ey;
                f[0] = __builtin_fmaf(ec, dx, es * dy);
                f[1] = __builtin_fmaf(ec, dy, -(es * dx));
                f[2] = wrap_angle(A.st.yaw[h] - A.st.yaw[g]);
                f[3] = __builtin_fmaf(ec, A.st.vx[h], es * A.st.vy[h]);
                f[4] = __builtin_fmaf(ec, A.st.vy[h], -(es * A.st.vx[h]));
                f[5] = A.st.length[h];
                f[6] = A.st.width[h];
                f[7] = 1.f;
            }
            for (int c = 0; c < 8; ++c)
                of[8L * j + c] = f[c];
        }
    }

    // ---- keys ----
    uint32_t key[kObsKeys];
    int nvalid_local = 0;
#pragma unroll
    for (int r = 0; r < kObsKeys; ++r) {
        const int j = tid + kObsThreads * r;
        uint32_t kk = kNoKey;
        if (ego_valid && j < P && A.rg.valid[p0 + j])
            kk = topk_key(A.rg.x[p0 + j], A.rg.y[p0 + j], ex, ey);
        key[r] = kk;
        nvalid_local += kk != kNoKey;
    }
    int nvalid;
    (void)block_exclusive(nvalid_local, wtot, &nvalid);
    const int kk = min(A.k, nvalid);

    // ---- radix select of the kk-th smallest key (rank kk-1) ----
    uint32_t prefix = 0, pmask = 0;
    int rank = kk - 1;
    const int shifts[3] = {21, 10, 0};
    const int widths[3] = {11, 11, 10};
    int *myhist = hist + kHistBins * (tid & (kHistCopies - 1));
    for (int pass = 0; pass < 3 && kk > 0; ++pass) {
        const int sh = shifts[pass], nb = 1 << widths[pass];
        for (int b = tid; b < kHistCopies * kHistBins; b += kObsThreads)
            hist[b] = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kObsKeys; ++r)
            if (key[r] != kNoKey && (key[r] & pmask) == prefix)
                atomicAdd(&myhist[(key[r] >> sh) & (nb - 1)], 1);
        __syncthreads();
        // find the bin holding `rank`: per-thread bin groups (copies summed),
        // then a block scan
        const int per = nb / kObsThreads > 0 ? nb / kObsThreads : 1;
        const int b0 = tid * per;
        int cnt = 0;
        if (b0 < nb)
            for (int b = b0; b < b0 + per; ++b)
                for (int c = 0; c < kHistCopies; ++c)
                    cnt += hist[kHistBins * c + b];
        int total;
        int before = block_exclusive(b0 < nb ? cnt : 0, wtot, &total);
        if (b0 < nb && rank >= before && rank < before + cnt) {
            int acc = before;
            for (int b = b0; b < b0 + per; ++b) {
                int hb = 0;
                for (int c = 0; c < kHistCopies; ++c)
                    hb += hist[kHistBins * c + b];
                if (rank < acc + hb) {
                    sh_bin = b;
                    sh_before = acc;
                    break;
                }
                acc += hb;
            }
        }
        __syncthreads();
        prefix |= (uint32_t)sh_bin << sh;
        pmask |= (uint32_t)(nb - 1) << sh;
        rank -= sh_before;
        __syncthreads();
    }
    const uint32_t kth = prefix;   // the kk-th smallest key (when kk > 0)

    // ---- compaction: keys < kth, then the lowest-index keys == kth ----
    int nless_local = 0, nle_local = 0;
#pragma unroll
    for (int r = 0; r < kObsKeys; ++r) {
        nless_local += (kk > 0 && key[r] < kth);
        nle_local += (kk > 0 && key[r] <= kth);
    }
    int nless, nle;
    (void)block_exclusive(nless_local, wtot, &nless);
    const int le_before = block_exclusive(nle_local, wtot, &nle);
    const int need_eq = kk - nless;
    if (nle == kk) {
        // no tie to break at the k-th key: every key <= kth is selected; each
        // thread writes its keys at its exclusive prefix (order is irrelevant:
        // the list is sorted below)
        int pos = le_before;
#pragma unroll
        for (int r = 0; r < kObsKeys; ++r)
            if (kk > 0 && key[r] <= kth)
                sel[pos++] = ((uint64_t)key[r] << 32) | (uint32_t)(tid + kObsThreads * r);
    } else {
        // more keys equal the k-th than are needed: the lowest indices win,
        // ranked in index order (j = tid + 1024 r) one round r at a time
        if (tid == 0)
            sh_count = 0;
        __syncthreads();
        int eq_seen = 0;   // equal keys at lower index, summed over earlier rounds
        for (int r = 0; r < kObsKeys; ++r) {
            const bool eq = kk > 0 && key[r] == kth;
            int tot;
            const int ex_rank = block_exclusive(eq ? 1 : 0, wtot, &tot);
            const bool take = (kk > 0 && key[r] < kth) || (eq && eq_seen + ex_rank < need_eq);
            if (take) {
                const int pos = atomicAdd(&sh_count, 1);
                sel[pos] = ((uint64_t)key[r] << 32) | (uint32_t)(tid + kObsThreads * r);
            }
            eq_seen += tot;
        }
    }
    __syncthreads();
    // pad to a power of two and sort ascending
    int m = 1;
    while (m < kk)
        m <<= 1;
    for (int i = kk + tid; i < m; i += kObsThreads)
        sel[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= m; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < m; i += kObsThreads) {
                const int partner = i ^ stride;
                if (partner > i) {
                    const bool up = (i & size) == 0;
                    const uint64_t a = sel[i], b = sel[partner];
                    if ((a > b) == up) {
                        sel[i] = b;
                        sel[partner] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // ---- outputs ----
    for (int r = tid; r < A.k; r += kObsThreads) {
        int idx = -1;
        float f[4] = {0.f, 0.f, 0.f, 0.f};
        if (r < kk) {
            idx = (int)(uint32_t)(sel[r] & 0xffffffffu);
            const int h = p0 + idx;
            const float dx = A.rg.x[h] - ex, dy = A.rg.y[h] - ey;
            f[0] = __builtin_fmaf(ec, dx, es * dy);
            f[1] = __builtin_fmaf(ec, dy, -(es * dx));
            f[2] = __builtin_fmaf(ec, A.rg.dir_x[h], es * A.rg.dir_y[h]);
            f[3] = __builtin_fmaf(ec, A.rg.dir_y[h], -(es * A.rg.dir_x[h]));
        }
        A.rg_idx[out0 + r] = idx;
        if (A.rg_feat)
            for (int c = 0; c < 4; ++c)
                A.rg_feat[4 * (out0 + r) + c] = f[c];
    }
}

void launch_observe(const wm_batch &b, const ObserveArgs &a, int rows, hipStream_t st)
{
    hipLaunchKernelGGL(k_observe, dim3(b.num_scenarios * a.E, rows), dim3(kObsThreads), 0, st, a);
}

} // namespace wm
