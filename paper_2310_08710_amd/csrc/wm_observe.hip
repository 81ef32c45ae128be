// wm_observe.hip -- default observation (Sec. 3.2): objects in the ego frame
// and the k road points nearest to the ego, exact, ascending by
// (binary32 squared distance, index).
//
// One 1024-thread work-group per (row, scenario, ego); two fit on a CU.  A
// scenario's road graph is read once per ego (point j by thread j % 1024).
// The keys are non-negative floats, whose bit patterns order like their
// values.
//   1. Every 16th point is sampled; a histogram of the samples' top bits
//      (exponent and three mantissa bits) gives a bound U below which about
//      1.5 k keys should lie.
//   2. Every key is computed once; those below U are appended to an LDS list
//      (wave ballots, one atomic per wave and round that has any).  If the
//      list holds at least k keys and did not overflow, the rest are never
//      touched again; otherwise (rarely) every point is a candidate, its key
//      recomputed from the road graph.
//   3. A histogram of the candidates' first digit (key bits 19..30: exponent
//      and four mantissa bits, 4096 bins) locates the bin b holding the k-th
//      key; every candidate below that bin is selected.
//   4. The keys of bin b (rarely more than a few hundred; otherwise the next
//      digits narrow it first) are ranked among themselves by (key, index),
//      and the lowest ones fill the last places.
//   5. The selected keys below bin b are scattered into LDS grouped by their
//      bin, whose output range is known from the histogram's prefix sum, and
//      each one's place is the start of its bin plus the number of keys of
//      that bin that precede it.
//   6. The places are collected in LDS and the outputs written in place
//      order (coalesced).
// No sorting network: twelve work-group barriers per ego on the list path.
#include "wm_device.h"
#include "wm_internal.h"

namespace wm {

constexpr int kObsThreads = 1024;
constexpr int kObsKeys = WM_MAX_OBSERVE_POINTS / kObsThreads;  // 32
constexpr uint32_t kNoKey = 0xffffffffu;                        // invalid point
constexpr uint32_t kAllKeys = 0x80000000u;                      // above every valid key
constexpr int kBins = 4096;                                     // first digit: key bits 19..30
constexpr int kDigitShift = 19;
constexpr int kHistCopies = 1;
constexpr int kBinsPerThread = kBins / kObsThreads;
constexpr int kSampleBins = 2048;                               // sample digit: key bits 20..30
constexpr int kSampleShift = 20;
constexpr int kCandCap = 1024;                                  // boundary keys ranked directly
constexpr int kListCap = 3072;                                  // candidates compacted into LDS
static_assert(kListCap >= WM_MAX_TOPK, "the list's key array then holds the output order");

__device__ __forceinline__ uint32_t topk_key(float qx, float qy, float ex, float ey)
{
    const float dx = qx - ex, dy = qy - ey;
    const float xx = dx * dx, yy = dy * dy;  // no contraction: fl(fl(dx*dx) + fl(dy*dy))
    return __float_as_uint(xx + yy) & 0x7fffffffu;
}

// Block-wide exclusive prefix of a per-thread count; returns the exclusive
// prefix and writes the block total to *total.  Two barriers.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t *wtot, uint32_t *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = v;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(incl, d);
        if (lane >= d)
            incl += u;
    }
    if (lane == 63)
        wtot[w] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int i = 0; i < kObsThreads / 64; ++i) {
        off += (i < w) ? wtot[i] : 0u;
        tot += wtot[i];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// Number of entries of a[lo, hi) below `own`, eight loads in flight.
__device__ __forceinline__ int count_below(const uint64_t *a, int lo, int hi, uint64_t own)
{
    int c = 0, q = lo;
    for (; q + 8 <= hi; q += 8) {
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = a[q + u];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            c += v[u] < own;
    }
    for (; q < hi; ++q)
        c += a[q] < own;
    return c;
}

// Sum over the wave.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    for (int d = 32; d > 0; d >>= 1)
        v += __shfl_xor(v, d);
    return v;
}

struct TopkLds {
    int *hist;           // [kHistCopies][kBins] digit histograms; copy 0 then the scatter cursors
    int *base;           // [kBins + 1] exclusive prefix of the first-digit histogram
    uint64_t *sel;       // [WM_MAX_TOPK] selected keys below the boundary, grouped by bin
    uint64_t *cand;      // [kCandCap] keys of the boundary set
    uint32_t *wtot;      // [16] per-wave totals of block_exclusive
    int *sh;             // [4] bin, before, count, boundary-list length
    int *order;          // [WM_MAX_TOPK] the point at each output place
};

// Every point of the scenario as a candidate, its key recomputed from the
// road graph at each pass (the rare fallback): point j = tid + 1024 r.
struct AllKeys {
    const float *rx, *ry;
    const uint8_t *rv;
    int P;
    bool have;   // ego valid and P > 0
    float ex, ey;
    template <class F> __device__ __forceinline__ void each(F &&f) const
    {
        if (!have)
            return;
#pragma unroll 4
        for (int r = 0; r < kObsKeys; ++r) {
            // indices past the scenario's points are clamped to its last
            // point (an in-bounds load) and give no key
            const int j = (int)threadIdx.x + kObsThreads * r, jj = min(j, P - 1);
            const uint32_t kq = topk_key(rx[jj], ry[jj], ex, ey);
            f((j < P && rv[jj] != 0) ? kq : kNoKey, j, r);
        }
    }
};

// Candidates compacted into LDS: keys and scenario-local indices.
struct ListKeys {
    const uint32_t *key;
    const uint32_t *idx;
    int n;
    template <class F> __device__ __forceinline__ void each(F &&f) const
    {
        for (int i = threadIdx.x; i < n; i += kObsThreads)
            f(key[i], (int)idx[i], 0);
    }
};

// Selects the kk (>= 1, <= number of candidates) smallest candidates in
// (key, index) order into L.order[0, kk); every candidate not given is larger
// than every one given.  Returns false, having written nothing, when the boundary
// set is over kCandCap equal keys and the candidates are not AllKeys (whose
// fixed index order that case needs).  Work-group-wide; every thread calls it
// with the same arguments.
template <bool kReg, class Src>
__device__ __forceinline__ bool topk_select(const Src &src, int kk, const TopkLds &L, bool cleared)
{
    const int tid = threadIdx.x;
    if (!cleared) {
        __syncthreads();   // earlier readers of the LDS arrays are done
        for (int b = tid; b < kHistCopies * kBins; b += kObsThreads)
            L.hist[b] = 0;
        if (tid < 4)
            L.sh[tid] = 0;
        __syncthreads();
    }

    // ---- first digit: histogram, prefix, the bin holding the kk-th key ----
    int *myhist = L.hist + kBins * (tid % kHistCopies);
    src.each([&](uint32_t k, int, int) {
        if (k != kNoKey)
            atomicAdd(&myhist[k >> kDigitShift], 1);
    });
    __syncthreads();
    constexpr int BPT = kBinsPerThread;
    int c[BPT], csum = 0;   // this thread's bins BPT tid .. BPT tid + BPT - 1, copies summed
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        c[i] = 0;
        for (int cp = 0; cp < kHistCopies; ++cp)
            c[i] += L.hist[kBins * cp + BPT * tid + i];
        csum += c[i];
    }
    uint32_t tot;
    const int ex0 = (int)block_exclusive((uint32_t)csum, L.wtot, &tot);
    if (tid == 0)
        L.base[kBins] = (int)tot;
    int run = ex0;
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        // only this thread read its bins: they become its scatter cursors
        L.base[BPT * tid + i] = run;
        L.hist[BPT * tid + i] = run;
        if (run <= kk - 1 && kk - 1 < run + c[i]) {
            L.sh[0] = BPT * tid + i;
            L.sh[1] = run;
            L.sh[2] = c[i];
        }
        run += c[i];
    }
    __syncthreads();
    // block-uniform from here on (read into scalar registers)
    const int b1 = __builtin_amdgcn_readfirstlane(L.sh[0]);
    uint32_t prefix = (uint32_t)b1 << kDigitShift, pmask = ~0u << kDigitShift;
    int c_less = __builtin_amdgcn_readfirstlane(L.sh[1]);   // candidates below the boundary set: all selected
    int nB = __builtin_amdgcn_readfirstlane(L.sh[2]);       // candidates with (key & pmask) == prefix

    // ---- a boundary bin too large to rank directly: narrow it by the
    // next 10-bit digits ----
    if (nB > kCandCap) {
        for (int pass = 0; pass < 2 && nB > kCandCap; ++pass) {
            // the next 10 bits below the first digit, then the rest
            const int sh = pass == 0 ? kDigitShift - 10 : 0;
            const uint32_t dm = pass == 0 ? 1023u : (1u << (kDigitShift - 10)) - 1u;
            __syncthreads();
            for (int cp = 0; cp < kHistCopies; ++cp)
                L.hist[kBins * cp + tid] = 0;
            __syncthreads();
            src.each([&](uint32_t k, int, int) {
                if ((k & pmask) == prefix)   // never true for kNoKey: prefix < 2^31
                    atomicAdd(&myhist[(k >> sh) & dm], 1);
            });
            __syncthreads();
            int cnt = 0;
            for (int cp = 0; cp < kHistCopies; ++cp)
                cnt += L.hist[kBins * cp + tid];
            uint32_t t2;
            const int exb = (int)block_exclusive((uint32_t)cnt, L.wtot, &t2);
            const int rank = kk - 1 - c_less;
            if (rank >= exb && rank < exb + cnt) {
                L.sh[0] = tid;
                L.sh[1] = exb;
                L.sh[2] = cnt;
            }
            __syncthreads();
            prefix |= (uint32_t)__builtin_amdgcn_readfirstlane(L.sh[0]) << sh;
            pmask |= dm << sh;
            c_less += __builtin_amdgcn_readfirstlane(L.sh[1]);
            nB = __builtin_amdgcn_readfirstlane(L.sh[2]);
        }
        if (!kReg && nB > kCandCap)
            return false;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < BPT; ++i)
            L.hist[BPT * tid + i] = L.base[BPT * tid + i];
        if (tid == 0)
            L.sh[3] = 0;
        __syncthreads();
    }
    const int need = kk - c_less;   // places taken from the boundary set

    // ---- scatter the candidates below the boundary; collect the boundary
    // set (or, when it is too large, mark its members: bit r of eqm) ----
    const bool direct = nB <= kCandCap;
    uint32_t eqm = 0;
    src.each([&](uint32_t k, int j, int r) {
        // kNoKey is neither below prefix nor in the boundary set
        const uint64_t ent = ((uint64_t)k << 32) | (uint32_t)j;
        if (k < prefix)
            L.sel[atomicAdd(&L.hist[k >> kDigitShift], 1)] = ent;
        else if ((k & pmask) == prefix) {
            if (!kReg || direct)
                L.cand[atomicAdd(&L.sh[3], 1)] = ent;
            else
                eqm |= 1u << r;
        }
    });
    __syncthreads();

    // ---- the boundary set: rank among itself, keep the lowest `need` ----
    if (direct) {
        // on the last threads: the first ones rank the keys below the boundary
        for (int c = kObsThreads - 1 - tid; c < nB; c += kObsThreads) {
            const uint64_t own = L.cand[c];
            const int before = count_below(L.cand, 0, nB, own);
            if (before < need)
                L.order[c_less + before] = (int)(uint32_t)own;
        }
    } else if (kReg) {
        // every key of the boundary set is equal (all digits fixed): the
        // lowest indices win.  Index order is j = tid + 1024 r: round r
        // first, then wave, then lane; wave counts per round go through LDS.
        const int lane = tid & 63, wv = tid >> 6;
        // [round][wave] counts in the boundary-set array, which this path
        // never fills (its members are marked in eqm instead)
        static_assert(kObsKeys * (kObsThreads / 64) * sizeof(int) <= kCandCap * sizeof(uint64_t),
                      "per-round wave counts fit in the boundary-set array");
        int *wc = (int *)L.cand;
        for (int r = 0; r < kObsKeys; ++r) {
            const int cnt = __popcll(__ballot((eqm >> r) & 1u));
            if (lane == 0)
                wc[r * (kObsThreads / 64) + wv] = cnt;
        }
        __syncthreads();
        int rounds_before = 0;
        for (int r = 0; r < kObsKeys; ++r) {
            const uint64_t bal = __ballot((eqm >> r) & 1u);
            int waves_before = 0, round_tot = 0;
            for (int v = 0; v < kObsThreads / 64; ++v) {
                const int c = wc[r * (kObsThreads / 64) + v];
                round_tot += c;
                waves_before += v < wv ? c : 0;
            }
            if ((eqm >> r) & 1u) {
                const int rk = rounds_before + waves_before + __popcll(bal & ((1ull << lane) - 1ull));
                if (rk < need)
                    L.order[c_less + rk] = tid + kObsThreads * r;
            }
            rounds_before += round_tot;
        }
    }
    // ---- candidates below the boundary: start of the bin + rank inside it ----
    for (int i = tid; i < c_less; i += kObsThreads) {
        const uint64_t own = L.sel[i];
        const int d = (int)(own >> (32 + kDigitShift));
        const int start = L.base[d], end = d == b1 ? c_less : L.base[d + 1];
        L.order[start + count_below(L.sel, start, end, own)] = (int)(uint32_t)own;
    }
    return true;
}

__global__ __launch_bounds__(kObsThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_observe(ObserveArgs A,
                                                                                                   int rows)
{
    // Work item w = (s * rows + row) * E + e.  Work-groups are dispatched to
    // the eight XCDs in turn; each XCD takes a contiguous range of w, so the
    // egos and rows of one scenario share that XCD's L2 copy of its road graph.
    const long W = (long)rows * A.S * A.E;
    const long p = blockIdx.x, full = W / 8 * 8;
    const long w = p < full ? (p % 8) * (W / 8) + p / 8 : p;
    const int e = (int)(w % A.E);
    const long sr = w / A.E;
    const int row = (int)(sr % rows), s = (int)(sr / rows);
    const int slot = s * A.E + e;
    const long so = (long)row * A.n, orow = (long)row * A.S * A.E;

    // 72 KB: two work-groups fit on a CU
    __shared__ int hist[kHistCopies * kBins];
    __shared__ int base[kBins + 1];
    __shared__ uint64_t sel[WM_MAX_TOPK];
    __shared__ uint64_t cand[kCandCap];         // first the sample histogram
    __shared__ uint32_t lkey[kListCap], lidx[kListCap];
    static_assert(kSampleBins * sizeof(int) <= kCandCap * sizeof(uint64_t), "sample histogram overlays cand");
    int *hs = (int *)cand;                      // sample-digit histogram of the sampled keys
    __shared__ uint32_t wtot[kObsThreads / 64];
    __shared__ int sh[4];
    __shared__ uint32_t sh_bound, sh_nvalid, sh_nU;
    const TopkLds L{hist, base, sel, cand, wtot, sh, (int *)lkey};   // the list is done with when places are set
    const int tid = threadIdx.x;
    const int o0 = A.obj_off[s], N = A.obj_off[s + 1] - o0;
    const int p0 = A.rg_off[s], P = A.rg_off[s + 1] - p0;
    const int g = A.ego[slot];
    const bool ego_valid = A.st.valid[so + g];
    const float ex = A.st.x[so + g], ey = A.st.y[so + g], eyaw = A.st.yaw[so + g];
    float es, ec;
    sincosf(eyaw, &es, &ec);
    for (int b = tid; b < kSampleBins; b += kObsThreads)
        hs[b] = 0;
    for (int b = tid; b < kHistCopies * kBins; b += kObsThreads)
        hist[b] = 0;
    if (tid < 4)
        sh[tid] = 0;
    if (tid == 0) {
        sh_bound = kAllKeys;
        sh_nvalid = 0;
        sh_nU = 0;
    }

    // ---- objects in the ego frame ----
    if (A.obj_feat) {
        float *of = A.obj_feat + (orow + slot) * A.maxN * 8;
        for (int j = tid; j < A.maxN; j += kObsThreads) {
            float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const long h = so + o0 + j;
            if (ego_valid && j < N && A.st.valid[h]) {
                const float dx = A.st.x[h] - ex, dy = A.st.y[h] - ey;
                f[0] = __builtin_fmaf(ec, dx, es * dy);
                f[1] = __builtin_fmaf(ec, dy, -(es * dx));
                f[2] = wrap_angle(A.st.yaw[h] - eyaw);
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

    // ---- pass A: the sample (every 16th point) bounds the k-th key ----
    const float *rx = A.rg.x + p0, *ry = A.rg.y + p0;
    const uint8_t *rv = A.rg.valid + p0;
    const bool have = ego_valid && P > 0;
    __syncthreads();   // hs, hist and the counters are cleared
    if (have) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {   // 16 (tid + 1024 h) covers every multiple of 16 below 32768
            const int j = 16 * (tid + kObsThreads * h);
            if (j < P && rv[j])
                atomicAdd(&hs[topk_key(rx[j], ry[j], ex, ey) >> kSampleShift], 1);
        }
    }
    __syncthreads();
    const int s0 = hs[2 * tid], s1 = hs[2 * tid + 1];
    uint32_t ns;
    const int exs = (int)block_exclusive((uint32_t)(s0 + s1), wtot, &ns);
    // the ns samples stand for about 16 ns valid points: aim at 1.5 k' keys
    // below U, k' = min(k, 16 ns)
    const int k_est = min(A.k, 16 * (int)ns);
    const int want = (3 * k_est + 31) / 32 + 4;
    if (want < (int)ns && exs <= want - 1 && want - 1 < exs + s0 + s1)
        sh_bound = (uint32_t)(want - 1 < exs + s0 ? 2 * tid + 1 : 2 * tid + 2) << kSampleShift;
    __syncthreads();
    const uint32_t U = __builtin_amdgcn_readfirstlane(sh_bound);

    // ---- pass B: every key, once; those below U are appended to the list
    // (any order: the selection ranks by (key, index)), one list atomic per
    // wave and round that has any ----
    const int lane = tid & 63;
    int nv_local = 0;
    if (have) {
#pragma unroll 8
        for (int r = 0; r < kObsKeys; ++r) {
            if (kObsThreads * r >= P)   // block-uniform
                break;
            // indices past the scenario's points are clamped to its last
            // point (an in-bounds load) and give no key
            const int j = tid + kObsThreads * r, jj = min(j, P - 1);
            const uint32_t kq = topk_key(rx[jj], ry[jj], ex, ey);
            const bool v = j < P && rv[jj] != 0;
            nv_local += v;
            const bool in = v && kq < U;
            const uint64_t bal = __ballot(in);
            if (bal) {   // wave-uniform
                int base = 0;
                if (lane == 0)
                    base = (int)atomicAdd(&sh_nU, (uint32_t)__popcll(bal));
                const int at = __builtin_amdgcn_readfirstlane(base) + __popcll(bal & ((1ull << lane) - 1ull));
                if (in && at < kListCap) {
                    lkey[at] = kq;
                    lidx[at] = (uint32_t)j;
                }
            }
        }
    }
    const uint32_t nv_wave = wave_sum((uint32_t)nv_local);
    if (lane == 0)
        atomicAdd(&sh_nvalid, nv_wave);
    __syncthreads();
    const int nvalid = __builtin_amdgcn_readfirstlane(sh_nvalid);
    const int kk = min(A.k, nvalid);
    const int nU = __builtin_amdgcn_readfirstlane((int)sh_nU);

    // the list holds the nU smallest keys; it serves when that is at least
    // kk and fits (otherwise, rarely: the sample misled, or too many keys
    // share the bound's bin), every point is a candidate
    bool done = kk == 0;
    if (!done && nU >= kk && nU <= kListCap)
        done = topk_select<false>(ListKeys{lkey, lidx, nU}, kk, L, true);
    if (!done)
        topk_select<true>(AllKeys{A.rg.x + p0, A.rg.y + p0, A.rg.valid + p0, P, ego_valid && P > 0, ex, ey}, kk,
                          L, false);
    __syncthreads();

    // ---- outputs in place order (coalesced), then the padding ----
    const long out0 = (orow + slot) * (long)A.k;
    float *feat = A.rg_feat ? A.rg_feat + 4 * out0 : nullptr;
    const bool feat16 = ((uintptr_t)A.rg_feat & 15u) == 0;
    for (int r = tid; r < A.k; r += kObsThreads) {
        const int j = r < kk ? L.order[r] : -1;
        A.rg_idx[out0 + r] = j;
        if (feat) {
            float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j >= 0) {
                const int h = p0 + j;
                const float dx = A.rg.x[h] - ex, dy = A.rg.y[h] - ey;
                f.x = __builtin_fmaf(ec, dx, es * dy);
                f.y = __builtin_fmaf(ec, dy, -(es * dx));
                f.z = __builtin_fmaf(ec, A.rg.dir_x[h], es * A.rg.dir_y[h]);
                f.w = __builtin_fmaf(ec, A.rg.dir_y[h], -(es * A.rg.dir_x[h]));
            }
            if (feat16) {
                *(float4 *)(feat + 4L * r) = f;
            } else {
                feat[4L * r] = f.x;
                feat[4L * r + 1] = f.y;
                feat[4L * r + 2] = f.z;
                feat[4L * r + 3] = f.w;
            }
        }
    }
}

void launch_observe(const wm_batch &b, const ObserveArgs &a, int rows, hipStream_t st)
{
    const long blocks = (long)rows * b.num_scenarios * a.E;
    hipLaunchKernelGGL(k_observe, dim3((unsigned)blocks), dim3(kObsThreads), 0, st, a, rows);
}

} // namespace wm
