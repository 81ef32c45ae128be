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
#include <hip/hip_fp16.h>

#include <map>
#include <mutex>

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
constexpr int32_t kHandOver = -2;   // first rg_idx place of an ego left to the exact kernel
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

// The exact selection of one work item w = (s * rows + row) * E + e by a
// 1024-thread work-group over every point of the scenario: the path of the
// egos that the block-pruned kernel below hands over (boundary sets too large
// to rank directly, e.g. many equal keys at the k-th place).
__device__ __forceinline__ void observe_exact_item(const ObserveArgs &A, int rows, long w)
{
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

// ---------------------------------------------------------------------------
// Block-pruned selection.  Road points are consecutive along their polylines,
// so 32 consecutive points (a block) span a short stretch of road.  A
// work-group takes one scenario, a range of state rows and a range of egos;
// it first bounds every block (box of its valid points, rounded outwards to
// half precision, the valid count and a bit mask of the valid points) in
// LDS, then for each (row, ego):
//   1. lb / ub = binary32 key of the nearest / farthest point of the box;
//      rounding is monotone, so lb <= key <= ub for every valid point of the
//      block.  The histogram of ub weighted by the valid counts gives a bound
//      U with at least kk valid points below it: every selected key is below
//      U, and only blocks with lb < U hold candidates.
//   2. A 1024-bin histogram of the candidates' keys over the 8 octaves below
//      U (128 bins per octave; lower keys share bin 0) locates the bin b of
//      the kk-th key.
//   3. A second scan scatters the keys below bin b into their bins' output
//      ranges and collects bin b.  Each key's place is the start of its bin
//      plus its (key, index) rank inside it (bin b: among bin b); each
//      thread writes the outputs of the keys it ranked.
// Egos whose bin b holds more than kBndCap keys, or a lower bin more than
// kBinRankCap (many equal or nearly equal keys), are handed to the exact
// kernel above: their first rg_idx place is set to kHandOver and nothing else
// is written for them here.  Work-groups are small (four waves, 30 KB of LDS)
// so that four of them, each with its own ego, share a CU.
// ---------------------------------------------------------------------------
constexpr int kFastThreads = 256;
constexpr int kFastWaves = kFastThreads / 64;
constexpr int kBlockPts = 32;
// blocks start at multiples of 8 global points, so a scenario spans at most
// (P + 7) / 32 + 1 of them
constexpr int kMaxBlocks = (WM_MAX_OBSERVE_POINTS + 7 + kBlockPts - 1) / kBlockPts;   // 1025
constexpr int kBlocksPerThread = (kMaxBlocks + kFastThreads - 1) / kFastThreads;   // 5
constexpr int kUbBins = 256;                                        // bound digit: 8 bins per octave
constexpr int kUbShift = 20;
constexpr uint32_t kUbLow = 114u << 3;                              // bin 0: keys below 2^-13
constexpr int kUbPerThread = kUbBins / kFastThreads;                // 1
constexpr int kWinBins = 1024;                                      // window digit: 128 bins per octave
constexpr int kWinShift = 16;
constexpr int kWinPerThread = kWinBins / kFastThreads;              // 4
constexpr int kBndCap = 128;                                        // boundary-bin keys ranked directly
constexpr int kBinRankCap = 128;                                    // keys of a lower bin ranked by counting
constexpr int kPtsPerThread = 8;                                    // bounding pass: consecutive points per thread
constexpr int kBoundChunk = kFastThreads * kPtsPerThread;
constexpr int kBoundGroups = 4;                                     // bounding pass: groups loaded at once
static_assert(kBlockPts / kPtsPerThread == 4, "four threads per block");
constexpr int kGroupsPerPass = kFastThreads / kBlockPts;            // candidate blocks per round
constexpr int kBlockMinRows = 4;                                    // rows per ego for the block-pruned form
constexpr int kScanRounds = 16;                                     // rounds loaded at once, keys kept
constexpr int kRankPerThread = WM_MAX_TOPK / kFastThreads;          // keys below bin b per thread (c_less < 1024)
static_assert(kUbPerThread >= 1 && kWinPerThread >= 2 && kRankPerThread >= 1, "at most 256 threads");

// Block-wide exclusive prefix for kFastThreads threads (two barriers).
__device__ __forceinline__ uint32_t fast_exclusive(uint32_t v, uint32_t *wtot, uint32_t *total)
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
#pragma unroll
    for (int i = 0; i < kFastWaves; ++i) {
        off += (i < w) ? wtot[i] : 0u;
        tot += wtot[i];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

__device__ __forceinline__ uint32_t key_of_offsets(float dx, float dy)
{
    const float xx = dx * dx, yy = dy * dy;   // as topk_key: fl(fl(dx*dx) + fl(dy*dy))
    return __float_as_uint(xx + yy) & 0x7fffffffu;
}

// Half-precision bounds rounded outwards (toward -inf for a minimum, +inf
// for a maximum): the box only grows, so the bounds stay valid.
__device__ __forceinline__ uint32_t pack_down_up(float lo, float hi)
{
    const __half l = __float2half_rd(lo), h = __float2half_ru(hi);
    return (uint32_t)__half_as_ushort(l) | ((uint32_t)__half_as_ushort(h) << 16);
}

__device__ __forceinline__ float2 unpack_lo_hi(uint32_t v)
{
    return make_float2(__half2float(__ushort_as_half((unsigned short)(v & 0xffffu))),
                       __half2float(__ushort_as_half((unsigned short)(v >> 16))));
}

__device__ __forceinline__ void write_row(const ObserveArgs &A, long out0, int r, int j, int p0, float ex, float ey,
                                          float es, float ecs)
{
    A.rg_idx[out0 + r] = j;
    if (A.rg_feat) {
        float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j >= 0) {
            const int h = p0 + j;
            const float dx = A.rg.x[h] - ex, dy = A.rg.y[h] - ey;
            f.x = __builtin_fmaf(ecs, dx, es * dy);
            f.y = __builtin_fmaf(ecs, dy, -(es * dx));
            f.z = __builtin_fmaf(ecs, A.rg.dir_x[h], es * A.rg.dir_y[h]);
            f.w = __builtin_fmaf(ecs, A.rg.dir_y[h], -(es * A.rg.dir_x[h]));
        }
        float *feat = A.rg_feat + 4 * (out0 + r);
        if (((uintptr_t)A.rg_feat & 15u) == 0) {
            *(float4 *)feat = f;
        } else {
            feat[0] = f.x;
            feat[1] = f.y;
            feat[2] = f.z;
            feat[3] = f.w;
        }
    }
}

// four waves per SIMD: four work-groups of four waves per CU
__global__ __launch_bounds__(kFastThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_observe_blocks(
    ObserveArgs A, int rows, int row_chunk, int ego_chunk)
{
    // work-group p: (scenario, ego range, row range); the XCD remap keeps a
    // scenario's work-groups on one XCD (its road graph in that L2)
    const int nrc = (rows + row_chunk - 1) / row_chunk, nec = (A.E + ego_chunk - 1) / ego_chunk;
    const long W = (long)A.S * nrc * nec;
    const long p = blockIdx.x, full = W / 8 * 8;
    const long w = p < full ? (p % 8) * (W / 8) + p / 8 : p;
    const int rc = (int)(w % nrc);
    const int ec = (int)((w / nrc) % nec);
    const int s = (int)(w / ((long)nec * nrc));
    const int r0 = rc * row_chunk, r1 = min(rows, r0 + row_chunk);
    const int e0 = ec * ego_chunk, e1 = min(A.E, e0 + ego_chunk);

    __shared__ uint2 bbox[kMaxBlocks];           // half-precision (xmin, xmax), (ymin, ymax) of the valid points
    __shared__ uint8_t bcnt[kMaxBlocks];         // valid points of the block
    __shared__ uint32_t bmask[kMaxBlocks];       // bit i: point 32 b + i - lead is in the scenario and valid
    __shared__ uint32_t ubh[kUbBins];            // ub histogram weighted by valid counts
    __shared__ uint32_t whist[kWinBins / 2];     // window histogram, then the scatter cursors: 16-bit
                                                 // counters, bin b in word b % 512, half b / 512
    __shared__ uint16_t base[kWinBins + 2];      // window prefix
    __shared__ uint64_t sel[WM_MAX_TOPK];        // keys below bin b, grouped by bin
    __shared__ uint64_t cand[kBndCap];           // keys of bin b
    __shared__ uint16_t cblk[kMaxBlocks];        // candidate blocks
    __shared__ uint32_t wtot[kFastWaves];
    __shared__ int sh[8];
    uint16_t *whist16 = (uint16_t *)whist;
    uint16_t *order = whist16;                   // the point at each output place, after the scatter

    const int tid = threadIdx.x, lane = tid & 63;
    const int o0 = A.obj_off[s], N = A.obj_off[s + 1] - o0;
    const int p0 = A.rg_off[s], P = A.rg_off[s + 1] - p0;
    const float *rx = A.rg.x + p0, *ry = A.rg.y + p0;
    const uint8_t *rv = A.rg.valid + p0;
    const int p1 = p0 + P;
    const int gA = p0 & ~7, lead = p0 - gA;   // blocks start at multiples of 8 points
    const int NB = (P + lead + kBlockPts - 1) / kBlockPts;   // <= kMaxBlocks

    // ---- block boxes: eight consecutive points per thread (two 16-byte
    // loads of x and of y, one 8-byte load of the flags when the arrays are
    // aligned), four threads per block, kBoundGroups groups per thread in
    // flight.  Blocks start at multiples of 8 in the global arrays: block b
    // holds the scenario's points j = 32 b + i - lead, i < 32 ----
    int nvalid_local = 0;
    const bool vec = ((((uintptr_t)A.rg.x) | ((uintptr_t)A.rg.y)) & 15u) == 0 && (((uintptr_t)A.rg.valid) & 7u) == 0;
    for (int c0 = 0; c0 < P + lead; c0 += kBoundGroups * kBoundChunk) {
        float px[kBoundGroups][kPtsPerThread], py[kBoundGroups][kPtsPerThread];
        bool pv[kBoundGroups][kPtsPerThread];
#pragma unroll
        for (int gq = 0; gq < kBoundGroups; ++gq) {
            const int t0 = c0 + gq * kBoundChunk + kPtsPerThread * tid;   // offset from the aligned start
            const long g0 = (long)gA + t0;
            if (vec && g0 + kPtsPerThread <= (long)p1) {
                const float4 xa = *(const float4 *)(A.rg.x + g0), xb = *(const float4 *)(A.rg.x + g0 + 4);
                const float4 ya = *(const float4 *)(A.rg.y + g0), yb = *(const float4 *)(A.rg.y + g0 + 4);
                const uint2 vv = *(const uint2 *)(A.rg.valid + g0);
                px[gq][0] = xa.x; px[gq][1] = xa.y; px[gq][2] = xa.z; px[gq][3] = xa.w;
                px[gq][4] = xb.x; px[gq][5] = xb.y; px[gq][6] = xb.z; px[gq][7] = xb.w;
                py[gq][0] = ya.x; py[gq][1] = ya.y; py[gq][2] = ya.z; py[gq][3] = ya.w;
                py[gq][4] = yb.x; py[gq][5] = yb.y; py[gq][6] = yb.z; py[gq][7] = yb.w;
#pragma unroll
                for (int i = 0; i < kPtsPerThread; ++i) {
                    const int j = t0 + i - lead;
                    const uint32_t byte = ((i < 4 ? vv.x : vv.y) >> (8 * (i & 3))) & 0xffu;
                    pv[gq][i] = j >= 0 && byte != 0;
                }
            } else {
#pragma unroll
                for (int i = 0; i < kPtsPerThread; ++i) {
                    // indices outside the scenario are clamped into it (an
                    // in-bounds load) and count as invalid
                    const int j = t0 + i - lead, jj = min(max(j, 0), P - 1);
                    px[gq][i] = rx[jj];
                    py[gq][i] = ry[jj];
                    pv[gq][i] = j >= 0 && j < P && rv[jj] != 0;
                }
            }
        }
#pragma unroll
        for (int gq = 0; gq < kBoundGroups; ++gq) {
            const int t0 = c0 + gq * kBoundChunk + kPtsPerThread * tid;
            float xmn = __builtin_inff(), xmx = -__builtin_inff(), ymn = __builtin_inff(), ymx = -__builtin_inff();
            int cnt = 0;
            uint32_t bits = 0;
#pragma unroll
            for (int i = 0; i < kPtsPerThread; ++i) {
                bits |= (pv[gq][i] ? 1u : 0u) << i;
                if (pv[gq][i]) {
                    xmn = fminf(xmn, px[gq][i]);
                    xmx = fmaxf(xmx, px[gq][i]);
                    ymn = fminf(ymn, py[gq][i]);
                    ymx = fmaxf(ymx, py[gq][i]);
                    ++cnt;
                }
            }
#pragma unroll
            for (int d = 1; d < 4; d <<= 1) {
                xmn = fminf(xmn, __shfl_xor(xmn, d));
                xmx = fmaxf(xmx, __shfl_xor(xmx, d));
                ymn = fminf(ymn, __shfl_xor(ymn, d));
                ymx = fmaxf(ymx, __shfl_xor(ymx, d));
                cnt += __shfl_xor(cnt, d);
            }
            bits <<= kPtsPerThread * (tid & 3);
            bits |= __shfl_xor(bits, 1);
            bits |= __shfl_xor(bits, 2);
            const int blk = t0 / kBlockPts;
            if ((tid & 3) == 0 && blk < NB) {
                bbox[blk] = make_uint2(pack_down_up(xmn, xmx), pack_down_up(ymn, ymx));
                bcnt[blk] = (uint8_t)cnt;
                bmask[blk] = bits;
                nvalid_local += cnt;
            }
        }
    }
    const uint32_t nv_wave = wave_sum((uint32_t)nvalid_local);
    if (tid == 0)
        sh[7] = 0;
    __syncthreads();
    if (lane == 0)
        atomicAdd((uint32_t *)&sh[7], nv_wave);
    __syncthreads();
    const int nvalid = __builtin_amdgcn_readfirstlane(sh[7]);
    const int kk = min(A.k, nvalid);
    const bool obj_regs = A.obj_feat && N <= 2 * kFastThreads;

    for (int e = e0; e < e1; ++e) {
        const int slot = s * A.E + e;
        const int g = A.ego[slot];
        // the previous row's kk-th key and ego position bound this row's
        // (triangle inequality), while the ego's rows follow one another
        bool have_prev = false;
        float px_prev = 0.f, py_prev = 0.f;
        for (int row = r0; row < r1; ++row) {
            const long so = (long)row * A.n, orow = (long)row * A.S * A.E;
            const bool ego_valid = A.st.valid[so + g];
            const float ex = A.st.x[so + g], ey = A.st.y[so + g], eyaw = A.st.yaw[so + g];
            float ob[2][7];
            bool obv[2];
            if (obj_regs) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int j = tid + kFastThreads * u;
                    const long h = so + o0 + min(j, max(N - 1, 0));
                    obv[u] = j < N && A.st.valid[h];
                    ob[u][0] = A.st.x[h];
                    ob[u][1] = A.st.y[h];
                    ob[u][2] = A.st.yaw[h];
                    ob[u][3] = A.st.vx[h];
                    ob[u][4] = A.st.vy[h];
                    ob[u][5] = A.st.length[h];
                    ob[u][6] = A.st.width[h];
                }
            }
            float es, ecs;
            sincosf(eyaw, &es, &ecs);
            const int kq = ego_valid ? kk : 0;
            const long out0 = (orow + slot) * (long)A.k;
            bool handed = false;
            // the previous row's kk-th key (written by its ranking, read
            // before this row clears the flags)
            __syncthreads();
            const uint32_t kth_prev = (uint32_t)__builtin_amdgcn_readfirstlane(sh[7]);
            const bool hint = have_prev && kq > 0;
            have_prev = false;
            if (kq > 0) {
                uint32_t hintU = kAllKeys;
                if (hint) {
                    // every previous selected point is within d_prev + |dp| of
                    // the ego now; margins cover the binary32 roundings
                    const float dpx = ex - px_prev, dpy = ey - py_prev;
                    const float dp = sqrtf(dpx * dpx + dpy * dpy);
                    const float dprev = sqrtf(__uint_as_float(kth_prev));
                    const float ud = (dprev + dp) * 1.00001f + 1e-6f;
                    const float uk = ud * ud * 1.00001f;
                    const uint32_t ub = __float_as_uint(uk) + 1u;
                    hintU = (uk < 3.0e38f && ub < kAllKeys) ? ub : kAllKeys;
                }
                uint32_t U = kAllKeys;
                int NC = 0, bb = 0, c_less = 0, nB = 0;
                uint32_t kreg[kScanRounds];
                int R = 0;
                const int cb = tid / kBlockPts, bl = tid & (kBlockPts - 1);
                auto point_of = [&](int r) {   // point of round r, or -1
                    const int c = cb + kGroupsPerPass * r;
                    const int j = c < NC ? kBlockPts * (int)cblk[c] + bl - lead : -1;
                    return j < P ? j : -1;
                };
                auto valid_of = [&](int r) {   // the point of round r is valid
                    const int c = cb + kGroupsPerPass * r;
                    return c < NC && ((bmask[cblk[c]] >> bl) & 1u) != 0;
                };
                auto load_keys = [&](int rb) {
                    float qx[kScanRounds], qy[kScanRounds];
                    bool qv[kScanRounds];
#pragma unroll
                    for (int q = 0; q < kScanRounds; ++q) {
                        qv[q] = false;
                        qx[q] = qy[q] = 0.f;
                        if (rb + q < R) {   // work-group uniform
                            const int jj = max(point_of(rb + q), 0);
                            qx[q] = rx[jj];
                            qy[q] = ry[jj];
                            qv[q] = valid_of(rb + q);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < kScanRounds; ++q) {
                        const uint32_t key = key_of_offsets(qx[q] - ex, qy[q] - ey);
                        kreg[q] = qv[q] && key < U ? key : kNoKey;
                    }
                };
                uint32_t dlo = 0;
                auto bin_of = [&](uint32_t key) {
                    const uint32_t d = key >> kWinShift;
                    return (int)(d > dlo ? d - dlo : 0u);
                };
                uint32_t wc[kWinPerThread];
                bool found = false;
                // attempt 0 takes the hinted bound when there is one; a bound
                // with fewer than kq keys below it (never expected) is
                // replaced by the block bound
                for (int attempt = hint ? 0 : 1; attempt < 2; ++attempt) {
                    const bool use_hint = attempt == 0;
                    __syncthreads();   // the previous ego's or attempt's readers are done
#pragma unroll
                    for (int i = 0; i < kUbPerThread; ++i)
                        ubh[kUbPerThread * tid + i] = 0;
#pragma unroll
                    for (int i = 0; i < kWinPerThread / 2; ++i)
                        whist[(kWinPerThread / 2) * tid + i] = 0;
                    if (tid < 8)
                        sh[tid] = 0;
                    __syncthreads();
                    // ---- 1. block bounds; the bound U ----
                    uint32_t lb[kBlocksPerThread];
#pragma unroll
                    for (int i = 0; i < kBlocksPerThread; ++i) {
                        const int b = tid + kFastThreads * i;
                        lb[i] = kNoKey;
                        if (b < NB && bcnt[b]) {
                            const uint2 q = bbox[b];
                            const float2 qx = unpack_lo_hi(q.x), qy = unpack_lo_hi(q.y);
                            const float lx = qx.x - ex, hx = qx.y - ex, ly = qy.x - ey, hy = qy.y - ey;
                            const float cx = lx > 0.f ? lx : (hx < 0.f ? -hx : 0.f);
                            const float cy = ly > 0.f ? ly : (hy < 0.f ? -hy : 0.f);
                            lb[i] = key_of_offsets(cx, cy);
                            if (!use_hint) {
                                const uint32_t ubk =
                                    key_of_offsets(fmaxf(fabsf(lx), fabsf(hx)), fmaxf(fabsf(ly), fabsf(hy)));
                                const uint32_t d = ubk >> kUbShift;
                                const uint32_t bin = d <= kUbLow ? 0u : min(d - kUbLow, (uint32_t)(kUbBins - 1));
                                atomicAdd(&ubh[bin], (uint32_t)bcnt[b]);
                            }
                        }
                    }
                    if (use_hint) {
                        U = hintU;
                    } else {
                        __syncthreads();
                        uint32_t uc[kUbPerThread], usum = 0;
#pragma unroll
                        for (int i = 0; i < kUbPerThread; ++i) {
                            uc[i] = ubh[kUbPerThread * tid + i];
                            usum += uc[i];
                        }
                        uint32_t utot;
                        uint32_t run = fast_exclusive(usum, wtot, &utot);
#pragma unroll
                        for (int i = 0; i < kUbPerThread; ++i) {
                            if (run <= (uint32_t)(kq - 1) && (uint32_t)(kq - 1) < run + uc[i])
                                sh[0] = kUbPerThread * tid + i;
                            run += uc[i];
                        }
                        __syncthreads();
                        // the upper edge of that bin (the top bin is open: no bound)
                        const int ubin = __builtin_amdgcn_readfirstlane(sh[0]);
                        U = ubin == kUbBins - 1 ? kAllKeys : ((uint32_t)ubin + kUbLow + 1u) << kUbShift;
                    }

                    // ---- candidate blocks: lb < U ----
#pragma unroll
                    for (int i = 0; i < kBlocksPerThread; ++i) {
                        const bool in = lb[i] < U;
                        const uint64_t bal = __ballot(in);
                        if (bal) {
                            int at0 = 0;
                            if (lane == 0)
                                at0 = atomicAdd(&sh[1], __popcll(bal));
                            const int at =
                                __builtin_amdgcn_readfirstlane(at0) + __popcll(bal & ((1ull << lane) - 1ull));
                            if (in)
                                cblk[at] = (uint16_t)(tid + kFastThreads * i);
                        }
                    }
                    __syncthreads();
                    NC = __builtin_amdgcn_readfirstlane(sh[1]);
                    const uint32_t dU = (U - 1u) >> kWinShift;
                    dlo = dU > (uint32_t)(kWinBins - 1) ? dU - (uint32_t)(kWinBins - 1) : 0u;
                    // candidate c of round r is block cblk[c], c = tid / 32 + 8 r;
                    // kScanRounds rounds are loaded at once and their keys kept
                    R = (NC + kGroupsPerPass - 1) / kGroupsPerPass;

                    // ---- 2. window histogram of the candidates' keys ----
                    for (int rb = 0; rb < R; rb += kScanRounds) {
                        load_keys(rb);
#pragma unroll
                        for (int q = 0; q < kScanRounds; ++q)
                            if (kreg[q] != kNoKey) {
                                const int bin = bin_of(kreg[q]);
                                atomicAdd(&whist[bin & (kWinBins / 2 - 1)], 1u << (16 * (bin / (kWinBins / 2))));
                            }
                    }
                    __syncthreads();
                    uint32_t wsum = 0;
#pragma unroll
                    for (int i = 0; i < kWinPerThread; ++i) {
                        const int bin = kWinPerThread * tid + i;
                        wc[i] = whist16[2 * (bin & (kWinBins / 2 - 1)) + bin / (kWinBins / 2)];
                        wsum += wc[i];
                    }
                    uint32_t wt;
                    uint32_t wrun = fast_exclusive(wsum, wtot, &wt);
                    if ((int)wt < kq)   // work-group uniform: too few keys below the hinted bound
                        continue;
                    if (tid == 0)
                        base[kWinBins] = (uint16_t)wt;
#pragma unroll
                    for (int i = 0; i < kWinPerThread; ++i) {
                        const int bin = kWinPerThread * tid + i;
                        base[bin] = (uint16_t)wrun;
                        // only this thread read this bin: it becomes its cursor
                        whist16[2 * (bin & (kWinBins / 2 - 1)) + bin / (kWinBins / 2)] = (uint16_t)wrun;
                        if (wrun <= (uint32_t)(kq - 1) && (uint32_t)(kq - 1) < wrun + wc[i]) {
                            sh[2] = bin;
                            sh[3] = (int)wrun;
                            sh[4] = (int)wc[i];
                        }
                        wrun += wc[i];
                    }
                    __syncthreads();
                    bb = __builtin_amdgcn_readfirstlane(sh[2]);
                    c_less = __builtin_amdgcn_readfirstlane(sh[3]);
                    nB = __builtin_amdgcn_readfirstlane(sh[4]);
                    found = true;
                    break;
                }
                // a bin below bb too large to rank by counting
#pragma unroll
                for (int i = 0; i < kWinPerThread; ++i)
                    if (kWinPerThread * tid + i < bb && wc[i] > (uint32_t)kBinRankCap)
                        sh[6] = 1;
                handed = !found || nB > kBndCap;
                if (!handed) {
                    // ---- 3. scatter below bb, collect bb (the keys are still
                    // in registers when one load pass covered every round) ----
                    for (int rb = 0; rb < R; rb += kScanRounds) {
                        if (R > kScanRounds)
                            load_keys(rb);
                        // every place is claimed before any is written, so
                        // the claims are in flight together
                        uint32_t at[kScanRounds];
#pragma unroll
                        for (int q = 0; q < kScanRounds; ++q) {
                            at[q] = 0xffffffffu;
                            if (kreg[q] != kNoKey) {
                                const int bin = bin_of(kreg[q]);
                                if (bin < bb) {
                                    const int sh16 = 16 * (bin / (kWinBins / 2));
                                    at[q] = (atomicAdd(&whist[bin & (kWinBins / 2 - 1)], 1u << sh16) >> sh16) & 0xffffu;
                                } else if (bin == bb) {
                                    at[q] = 0x10000u | (uint32_t)atomicAdd(&sh[5], 1);
                                }
                            }
                        }
#pragma unroll
                        for (int q = 0; q < kScanRounds; ++q)
                            if (at[q] != 0xffffffffu) {
                                const uint64_t ent = ((uint64_t)kreg[q] << 32) | (uint32_t)point_of(rb + q);
                                if (at[q] & 0x10000u)
                                    cand[at[q] & 0xffffu] = ent;
                                else
                                    sel[at[q]] = ent;
                            }
                    }
                    __syncthreads();
                    handed = __builtin_amdgcn_readfirstlane(sh[6]) != 0;
                    if (!handed) {
                        // ---- places (the point at each place goes to
                        // `order`, over the cursors, which are done with);
                        // the kk-th key is kept for the next row ----
                        const int need = kq - c_less;
                        for (int c = tid; c < nB; c += kFastThreads) {
                            const uint64_t own = cand[c];
                            const int before = count_below(cand, 0, nB, own);
                            if (before < need)
                                order[c_less + before] = (uint16_t)(uint32_t)own;
                            if (before == need - 1)
                                sh[7] = (int)(uint32_t)(own >> 32);
                        }
                        uint64_t own[kRankPerThread];
                        int st[kRankPerThread], en[kRankPerThread];
#pragma unroll
                        for (int u = 0; u < kRankPerThread; ++u) {
                            const int i = tid + kFastThreads * u;
                            own[u] = i < c_less ? sel[i] : 0;
                        }
#pragma unroll
                        for (int u = 0; u < kRankPerThread; ++u) {
                            const int bin = bin_of((uint32_t)(own[u] >> 32));
                            st[u] = base[bin];
                            en[u] = base[bin + 1];
                        }
#pragma unroll
                        for (int u = 0; u < kRankPerThread; ++u)
                            if (tid + kFastThreads * u < c_less)
                                order[st[u] + count_below(sel, st[u], en[u], own[u])] = (uint16_t)(uint32_t)own[u];
                        __syncthreads();
                        have_prev = true;
                        px_prev = ex;
                        py_prev = ey;
                    }
                }
            }
            if (handed) {
                if (tid == 0)
                    A.rg_idx[out0] = kHandOver;
                continue;
            }
            // ---- outputs in place order, then the padding, all rows of a
            // thread together ----
#pragma unroll
            for (int u = 0; u < WM_MAX_TOPK / kFastThreads; ++u) {
                const int r = tid + kFastThreads * u;
                if (r < A.k)
                    write_row(A, out0, r, r < kq ? (int)order[r] : -1, p0, ex, ey, es, ecs);
            }
            // ---- objects in the ego frame ----
            if (A.obj_feat) {
                float *of = A.obj_feat + (orow + slot) * A.maxN * 8;
                const bool of16 = ((uintptr_t)A.obj_feat & 15u) == 0;
                for (int j = tid; j < A.maxN; j += kFastThreads) {
                    float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    float o[7];
                    bool ov;
                    if (obj_regs) {
                        // j = tid or tid + kFastThreads: the registers loaded for this row
                        const int u = j < kFastThreads ? 0 : 1;
#pragma unroll
                        for (int c = 0; c < 7; ++c)
                            o[c] = u == 0 ? ob[0][c] : ob[1][c];
                        ov = u == 0 ? obv[0] : obv[1];
                    } else {
                        const long h = so + o0 + min(j, max(N - 1, 0));
                        ov = j < N && A.st.valid[h];
                        o[0] = A.st.x[h];
                        o[1] = A.st.y[h];
                        o[2] = A.st.yaw[h];
                        o[3] = A.st.vx[h];
                        o[4] = A.st.vy[h];
                        o[5] = A.st.length[h];
                        o[6] = A.st.width[h];
                    }
                    if (ego_valid && j < N && ov) {
                        const float dx = o[0] - ex, dy = o[1] - ey;
                        f[0] = __builtin_fmaf(ecs, dx, es * dy);
                        f[1] = __builtin_fmaf(ecs, dy, -(es * dx));
                        f[2] = wrap_angle(o[2] - eyaw);
                        f[3] = __builtin_fmaf(ecs, o[3], es * o[4]);
                        f[4] = __builtin_fmaf(ecs, o[4], -(es * o[3]));
                        f[5] = o[5];
                        f[6] = o[6];
                        f[7] = 1.f;
                    }
                    if (of16) {
                        *(float4 *)(of + 8L * j) = make_float4(f[0], f[1], f[2], f[3]);
                        *(float4 *)(of + 8L * j + 4) = make_float4(f[4], f[5], f[6], f[7]);
                    } else {
                        for (int c = 0; c < 8; ++c)
                            of[8L * j + c] = f[c];
                    }
                }
            }
        }
    }
}

// Every work item with the exact selection, one 1024-thread work-group per
// item: the form for few rows per ego (one state row), where the
// block-pruned kernel would bound a scenario's blocks for one or two
// observations.  Work-groups are dispatched to the eight XCDs in turn; each
// XCD takes a contiguous range of items, so the egos of one scenario share
// that XCD's L2 copy of its road graph.
__global__ __launch_bounds__(kObsThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_observe_each(ObserveArgs A,
                                                                                                        int rows)
{
    const long W = (long)rows * A.S * A.E;
    const long p = blockIdx.x, full = W / 8 * 8;
    observe_exact_item(A, rows, p < full ? (p % 8) * (W / 8) + p / 8 : p);
}

// The egos the block-pruned kernel marked (rg_idx of their first place set to
// kHandOver) get the exact selection over every point: each work-group reads
// the marks of 1024 consecutive work items and runs the marked ones in turn.
__global__ __launch_bounds__(kObsThreads) void k_observe_exact(ObserveArgs A, int rows)
{
    __shared__ int marked[kObsThreads];
    __shared__ int nmarked;
    const long W = (long)rows * A.S * A.E;
    for (long c0 = (long)blockIdx.x * kObsThreads; c0 < W; c0 += (long)gridDim.x * kObsThreads) {
        if (threadIdx.x == 0)
            nmarked = 0;
        __syncthreads();
        const long w = c0 + threadIdx.x;
        if (w < W) {
            const int e = (int)(w % A.E);
            const long sr = w / A.E;
            const int row = (int)(sr % rows), s = (int)(sr / rows);
            const long out0 = ((long)row * A.S * A.E + (long)s * A.E + e) * A.k;
            if (A.rg_idx[out0] == kHandOver)
                marked[atomicAdd(&nmarked, 1)] = (int)threadIdx.x;
        }
        __syncthreads();
        const int nm = nmarked;
        for (int i = 0; i < nm; ++i) {
            observe_exact_item(A, rows, c0 + marked[i]);
            __syncthreads();
        }
    }
}

// Resident work-groups of the block-pruned kernel per device (queried once
// per device, so later calls, e.g. under graph capture, make no queries).
static long observe_slots()
{
    static std::mutex mu;
    static std::map<int, long> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end())
        return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_observe_blocks, kFastThreads, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long slots = (long)per_cu * (cus < 1 ? 1 : cus);
    cache[dev] = slots;
    return slots;
}

void launch_observe(const wm_batch &b, const ObserveArgs &a, int rows, hipStream_t st)
{
    // Work-groups of the block-pruned kernel.  Each bounds its scenario's
    // blocks once for all of its (ego, row) pairs and runs an ego's rows in
    // order (each row's bound then comes from the previous one), so a
    // work-group takes as many observations as leave about four work-groups
    // per resident slot: consecutive rows of one ego, or, with fewer rows
    // than that, all rows of several egos.  Calls of fewer than
    // kBlockMinRows rows bound the blocks for too few observations: they
    // take the block form only when there are at least two observations per
    // resident slot (one work-group per slot, each bounding once for several
    // egos), the form with one work-group per observation otherwise.
    const long S = b.num_scenarios;
    const long items = (long)rows * S * a.E;
    const long slots = items >= 2 ? observe_slots() : 1;
    if (rows < kBlockMinRows && items < 2 * slots) {
        hipLaunchKernelGGL(k_observe_each, dim3((unsigned)items), dim3(kObsThreads), 0, st, a, rows);
        return;
    }
    long per = rows < kBlockMinRows ? items / slots : items / (4 * slots);
    if (per < 1)
        per = 1;
    int row_chunk = rows, ego_chunk = 1;
    if (rows < kBlockMinRows) {
        const long ec = per / rows;
        ego_chunk = (int)(ec < a.E ? ec : a.E);
        if (ego_chunk < 1)
            ego_chunk = 1;
    } else if (rows >= per) {
        row_chunk = (int)per;
    } else {
        const long ec = per / rows;
        ego_chunk = (int)(ec < a.E ? ec : a.E);
        if (ego_chunk < 1)
            ego_chunk = 1;
    }
    const long nrc = (rows + row_chunk - 1) / row_chunk, nec = (a.E + ego_chunk - 1) / ego_chunk;
    hipLaunchKernelGGL(k_observe_blocks, dim3((unsigned)(S * nrc * nec)), dim3(kFastThreads), 0, st, a, rows,
                       row_chunk, ego_chunk);
    long groups = (items + kObsThreads - 1) / kObsThreads;
    if (groups > 2048)
        groups = 2048;
    hipLaunchKernelGGL(k_observe_exact, dim3((unsigned)groups), dim3(kObsThreads), 0, st, a, rows);
}

} // namespace wm
