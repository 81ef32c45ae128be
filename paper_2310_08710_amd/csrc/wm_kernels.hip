// wm_kernels.hip -- HIP kernels of the simulator hot path for gfx950.
//
// Kernels (all float32):
//   k_compact_edges  road-graph preparation: valid road-edge points of each
//                    scenario packed in index order, padded to whole chunks
//   k_build_units    work-unit table (scenario, object slice) in descending
//                    cost order for the persistent rollout kernel
//   k_dynamics       one plain step: bicycle forward / playback / frozen (+ log divergence)
//   k_inverse        bicycle inverse kinematics
//   k_overlap        plain collision metric (+ optional margin matrix)
//   k_offroad        plain off-road metric
//   k_rollout        persistent fused rollout: T steps of dynamics + all metrics
//                    + training loss + checkpoints per work unit
//   k_loss_reduce    deterministic per-scenario sum of the loss partials
//   k_observe, k_rollout_backward live in their own sections below.
#include <map>
#include <mutex>
#include <tuple>

#include "wm_device.h"
#include "wm_internal.h"

namespace wm {

// ---------------------------------------------------------------------------
// Road-edge compaction into the workspace stream (layout in wm_internal.h,
// struct Edges): the valid road edges of scenario s in index order, chunked
// as x[], y[], qq[] columns of kEdgeChunk points, plus their directions, original indices, count and
// the largest qq (it bounds the rounding of the scan's expanded distance).
// ---------------------------------------------------------------------------
// One work-group per scenario.  A round covers PPT sub-rounds of BT
// consecutive points (sub-round k: point j0 + k BT + thread); the waves'
// ballot counts of every sub-round are prefix-summed in (sub-round, wave)
// order by the first wave, so a round costs two barriers and every load is
// coalesced.  A scenario of 30,000 points takes four rounds.
template <int BT, int PPT>
__global__ __launch_bounds__(BT) void k_compact_edges(const int32_t *__restrict__ rg_off, wm_roadgraph rg, Edges E)
{
    constexpr int NW = BT / 64, NC = PPT * NW;
    static_assert(NC <= 128, "two counts per lane of the first wave");
    __shared__ int cnt_k[NC], off_k[NC + 1];
    __shared__ unsigned int qqmax_bits;
    const int s = blockIdx.x;
    const int p0 = rg_off[s], p1 = rg_off[s + 1];
    const long base = edge_base(p0, s);                // first point slot of the scenario
    float *stream = E.stream + 3 * base;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0)
        qqmax_bits = 0u;
    __syncthreads();
    float my_max = 0.f;
    int run = 0;   // edges of the earlier rounds (the same in every thread)
    for (int j0 = p0; j0 < p1; j0 += BT * PPT) {
        uint64_t m[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int j = j0 + k * BT + threadIdx.x;
            m[k] = __ballot(j < p1 && rg.valid[j] && rg.type[j] == WM_TYPE_ROAD_EDGE);
            if (lane == 0)
                cnt_k[k * NW + w] = __popcll(m[k]);
        }
        __syncthreads();
        if (w == 0) {
            // exclusive prefix of the NC counts, two per lane
            const int a = 2 * lane < NC ? cnt_k[2 * lane] : 0;
            const int b = 2 * lane + 1 < NC ? cnt_k[2 * lane + 1] : 0;
            int incl = a + b;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int v = __shfl_up(incl, d);
                if (lane >= d)
                    incl += v;
            }
            const int excl = incl - a - b;
            if (2 * lane < NC)
                off_k[2 * lane] = excl;
            if (2 * lane + 1 < NC)
                off_k[2 * lane + 1] = excl + a;
            if (lane == 63)
                off_k[NC] = incl;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if ((m[k] >> lane) & 1ull) {
                const int j = j0 + k * BT + threadIdx.x;
                const int below =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(m[k] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m[k], 0));
                const int o = run + off_k[k * NW + w] + below;
                const float x = rg.x[j], y = rg.y[j];
                const float qq = __builtin_fmaf(y, y, x * x);
                float *ch = stream + kChunkFloats * (o / kChunk);
                ch[o % kChunk] = x;
                ch[kChunk + o % kChunk] = y;
                ch[2 * kChunk + qq_slot(o % kChunk)] = qq;
                E.dir[base + o] = make_float2(rg.dir_x[j], rg.dir_y[j]);
                E.idx[base + o] = j - p0;
                my_max = fmaxf(my_max, qq);
            }
        }
        run += off_k[NC];
    }
    __syncthreads();
    atomicMax(&qqmax_bits, __float_as_uint(my_max));   // qq >= 0: bit order = value order
    const int cnt = run;
    const int padded = (cnt + kChunk - 1) / kChunk * kChunk;
    for (int o = cnt + threadIdx.x; o < padded; o += BT) {
        float *ch = stream + kChunkFloats * (o / kChunk);
        ch[o % kChunk] = 0.f;
        ch[kChunk + o % kChunk] = 0.f;
        ch[2 * kChunk + qq_slot(o % kChunk)] = __builtin_inff();
        E.dir[base + o] = make_float2(0.f, 0.f);
        E.idx[base + o] = -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        E.count[s] = cnt;
        E.qqmax[s] = __uint_as_float(qqmax_bits);
    }
}

// ---------------------------------------------------------------------------
// Boxes of the compacted road edges: per block of 32 stream points and per
// chunk, the box of its edge points (padding excluded).  One work-group per
// scenario, one thread per chunk.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_edge_boxes(const int32_t *__restrict__ rg_off, Edges E)
{
    const int s = blockIdx.x;
    const long base = edge_base(rg_off[s], s);
    const int cnt = E.count[s];
    const int nch = (cnt + kChunk - 1) / kChunk;
    const float *stream = E.stream + 3 * base;
    for (int c = threadIdx.x; c < nch; c += blockDim.x) {
        const float4 *X = (const float4 *)(stream + (long)kChunkFloats * c);
        const float4 *Y = (const float4 *)(stream + (long)kChunkFloats * c + kChunk);
        float4 cb = make_float4(__builtin_inff(), -__builtin_inff(), __builtin_inff(), -__builtin_inff());
        for (int sb = 0; sb < kChunk / kBoxPts; ++sb) {
            float4 bb = make_float4(__builtin_inff(), -__builtin_inff(), __builtin_inff(), -__builtin_inff());
#pragma unroll
            for (int q = 0; q < kBoxPts / 4; ++q) {
                const int g4 = sb * (kBoxPts / 4) + q;
                const float4 xs = X[g4], ys = Y[g4];
                const float xv[4] = {xs.x, xs.y, xs.z, xs.w}, yv[4] = {ys.x, ys.y, ys.z, ys.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (kChunk * c + 4 * g4 + k < cnt) {
                        bb.x = fminf(bb.x, xv[k]);
                        bb.y = fmaxf(bb.y, xv[k]);
                        bb.z = fminf(bb.z, yv[k]);
                        bb.w = fmaxf(bb.w, yv[k]);
                    }
                }
            }
            E.box[base / kBoxPts + (kChunk / kBoxPts) * c + sb] = bb;
            cb = make_float4(fminf(cb.x, bb.x), fmaxf(cb.y, bb.y), fminf(cb.z, bb.z), fmaxf(cb.w, bb.w));
        }
        E.cbox[base / kChunk + c] = cb;
    }
}

// ---------------------------------------------------------------------------
// Work units of the persistent rollout: scenario s is cut into
// ceil(N_s / U) slices of U objects.  Unit ids are scenario-major
// (uoff[s] + slice); the queue holds them in descending cost order, a
// longest-first schedule.  Also resets the queue counter.  One block of 1024
// threads.
// ---------------------------------------------------------------------------
// Estimated cycles of one step of a unit of n objects with ep padded road
// edges (times 2): the off-road scan runs at a granularity of 16 objects per
// wave (64 lanes, 4 corners each) at about 2.5 instructions per corner and
// edge, the candidate rescans at about 100 per object, plus a fixed part for
// the barriers.  Only the order of the units depends on it; a term for the
// pair tests (n x N) ordered the ragged batch measurably worse.
__device__ __forceinline__ unsigned long long unit_cost(int n, unsigned long long ep)
{
    return 5ull * (unsigned long long)((n + 15) / 16) * ep + 200ull * n + 8000ull;
}

__global__ __launch_bounds__(1024) void k_build_units(const int32_t *__restrict__ obj_off,
                                                      const int32_t *__restrict__ ecount, int S, int U,
                                                      int32_t *__restrict__ uoff, int2 *__restrict__ units,
                                                      int32_t *__restrict__ counter)
{
    constexpr int NB = 1024;
    __shared__ int sh[1024];
    __shared__ unsigned long long maxcost;
    __shared__ int start[NB];
    __shared__ int carry;
    const int tid = threadIdx.x;
    if (tid == 0) {
        carry = 0;
        maxcost = 1;
    }
    start[tid] = 0;
    __syncthreads();
    // uoff: exclusive scan of units per scenario
    for (int s0 = 0; s0 < S; s0 += 1024) {
        const int s = s0 + tid;
        int nu = 0;
        if (s < S) {
            const int N = obj_off[s + 1] - obj_off[s];
            nu = (N + U - 1) / U;
        }
        sh[tid] = nu;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int v = tid >= d ? sh[tid - d] : 0;
            __syncthreads();
            sh[tid] += v;
            __syncthreads();
        }
        if (s < S)
            uoff[s] = carry + sh[tid] - nu;
        __syncthreads();
        if (tid == 1023)
            carry += sh[1023];
        __syncthreads();
    }
    const int total = carry;
    if (tid == 0) {
        uoff[S] = total;
        counter[0] = 0;
        counter[1] = total;
    }
    if (tid < 2 * kRollCountN)
        counter[kRollCounts + tid] = 0;
    // costs
    for (int s = tid; s < S; s += 1024) {
        const int N = obj_off[s + 1] - obj_off[s];
        const unsigned long long ep = ecount ? (unsigned long long)((ecount[s] + kChunk - 1) / kChunk * kChunk + kChunk)
                                             : (unsigned long long)kChunk;
        for (int sl = 0; sl * U < N; ++sl) {
            const unsigned long long c = unit_cost(min(U, N - sl * U), ep);
            atomicMax(&maxcost, c);
        }
    }
    __syncthreads();
    const unsigned long long mc = maxcost;
    for (int s = tid; s < S; s += 1024) {
        const int N = obj_off[s + 1] - obj_off[s];
        const unsigned long long ep = ecount ? (unsigned long long)((ecount[s] + kChunk - 1) / kChunk * kChunk + kChunk)
                                             : (unsigned long long)kChunk;
        for (int sl = 0; sl * U < N; ++sl) {
            const unsigned long long c = unit_cost(min(U, N - sl * U), ep);
            const int b = (int)((c * (NB - 1)) / mc);
            atomicAdd(&start[b], 1);
        }
    }
    __syncthreads();
    // exclusive scan in descending bucket order: bucket NB-1 first
    sh[tid] = start[NB - 1 - tid];
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = tid >= d ? sh[tid - d] : 0;
        __syncthreads();
        sh[tid] += v;
        __syncthreads();
    }
    const int excl = sh[tid] - start[NB - 1 - tid];
    __syncthreads();
    start[NB - 1 - tid] = excl;
    __syncthreads();
    for (int s = tid; s < S; s += 1024) {
        const int N = obj_off[s + 1] - obj_off[s];
        const unsigned long long ep = ecount ? (unsigned long long)((ecount[s] + kChunk - 1) / kChunk * kChunk + kChunk)
                                             : (unsigned long long)kChunk;
        for (int sl = 0; sl * U < N; ++sl) {
            const unsigned long long c = unit_cost(min(U, N - sl * U), ep);
            const int b = (int)((c * (NB - 1)) / mc);
            const int pos = atomicAdd(&start[b], 1);
            units[pos] = make_int2(s, sl);
        }
    }
}

// ---------------------------------------------------------------------------
// Shared per-unit pieces used by the plain and the fused kernels.  The
// objects of one scenario live in LDS (ObjLds, scenario-local index).
// ---------------------------------------------------------------------------
__device__ __forceinline__ Box lds_box(const ObjLds &L, int i)
{
    Box b;
    b.x = L.x[i];
    b.y = L.y[i];
    b.c = L.c[i];
    b.s = L.s[i];
    b.hl = 0.5f * L.len[i];
    b.hw = 0.5f * L.wid[i];
    return b;
}

__device__ __forceinline__ float sigmoidf(float z)
{
    return 1.0f / (1.0f + expf(-z));
}

// Overlap of slice objects i0 .. i0+Ns-1 against all N objects.  Thread
// (il = tid % U, part = tid / U) takes partners j = part, part + P, ...;
// per-thread maxima go to red[part * U + il].  When `loss` is set, the
// soft-overlap term of every pair (i, j > i) with a controlled member is
// added to *loss.  When `row` is set, margins / mask of row i are written.
__device__ __forceinline__ void overlap_partial(const ObjLds &L, int N, int i0, int Ns, int U, int P, float *red,
                                                float *loss, float *row_margin, uint8_t *row_mask)
{
    const int tid = threadIdx.x;
    const int il = tid % U, part = tid / U;
    if (part >= P)
        return;
    const int i = i0 + il;
    float mmax = kNoValue;
    if (il < Ns) {
        const bool vi = L.valid[i];
        const Box bi = lds_box(L, i);
        // every pair is evaluated (operands in index order) and the invalid
        // ones masked, so that the loop carries no branches
        for (int j = part; j < N; j += P) {
            const Box bj = lds_box(L, j);
            const float mm = sat_margin_ordered(bi, bj, i < j);   // sat_margin in index order
            const bool use = vi && j != i && L.valid[j];
            const float m = use ? mm : kNoValue;
            if (loss && use && j > i && (L.ctrl[i] || L.ctrl[j]))
                *loss += sigmoidf(m * (1.0f / kSoftScale));
            if (row_margin)
                row_margin[(long)il * N + j] = m;
            if (row_mask)
                row_mask[(long)il * N + j] = (uint8_t)(m > 0.f);
            mmax = fmaxf(mmax, m);
        }
    }
    red[part * U + il] = mmax;
}

// overlap_partial with each object's box packed in LDS as two float4, (x, y,
// cos, sin) and (half length, half width, valid, 0), written by the
// dynamics: two 16-byte reads per partner instead of seven, the same
// margins bit for bit.
__device__ __forceinline__ void overlap_partial_packed(const ObjLds &L, const float4 *obox, int N, int i0, int Ns,
                                                       int U, int P, float *red, float *loss)
{
    const int tid = threadIdx.x;
    const int il = tid % U, part = tid / U;
    if (part >= P)
        return;
    const int i = i0 + il;
    float mmax = kNoValue;
    if (il < Ns) {
        const float4 pi = obox[2 * i], qi = obox[2 * i + 1];
        const bool vi = qi.z != 0.f;
        const Box bi{pi.x, pi.y, pi.z, pi.w, qi.x, qi.y};
        for (int j = part; j < N; j += P) {
            const float4 pj = obox[2 * j], qj = obox[2 * j + 1];
            const Box bj{pj.x, pj.y, pj.z, pj.w, qj.x, qj.y};
            const float mm = sat_margin_ordered(bi, bj, i < j);
            const bool use = vi && j != i && qj.z != 0.f;
            const float m = use ? mm : kNoValue;
            if (loss && use && j > i && (L.ctrl[i] || L.ctrl[j]))
                *loss += sigmoidf(m * (1.0f / kSoftScale));
            mmax = fmaxf(mmax, m);
        }
    }
    red[part * U + il] = mmax;
}

// Per-split candidate lists of the off-road scan in LDS: for every split g
// and corner slot, the three smallest chunk minima and the first two chunks.
struct ScanLds {
    float4 *stage;  // one chunk stage per wave (kStageBytes each)
    float *b1, *b2, *b3;
    int *i1, *i2;
    int *full;      // corner slots that need the exact scan of every chunk
    int *nfull;
};

// p must be 16-byte aligned; waves = G * SL / 256.
__device__ __forceinline__ ScanLds carve_scan(void *p, int G, int SL)
{
    float4 *stage = (float4 *)p;
    float *f = (float *)((unsigned char *)p + (size_t)kStageBytes * (G * SL / 256));
    const int m = G * SL;
    int *fl = (int *)(f + 5 * m);
    return ScanLds{stage, f, f + m, f + 2 * m, (int *)(f + 3 * m), (int *)(f + 4 * m), fl, fl + SL};
}

constexpr size_t scan_lds_bytes(int G, int CW)
{
    return (size_t)kStageBytes * G * CW + (size_t)G * 256 * CW * 20 + (size_t)256 * CW * 4 + 16;
}

// Objects per group of the fused rollout's pruned scan (offroad_unit_pruned):
// a wave scans for the 4 kGroupObjects corners of a group at a time.
constexpr int kGroupObjects = 4;
// Road-edge chunks whose boxes (chunk and block boxes, 80 bytes per chunk)
// the fused rollout copies into LDS; a scenario with more reads them from
// global memory.
constexpr int kLdsBoxChunks = 256;
// Steps between renewals of the fused rollout's spatial order.
constexpr int kReorderSteps = 4;
// Objects per scenario up to which the fused rollout packs the boxes for
// its overlap (32 bytes of LDS per object).
constexpr int kPackedMaxN = 256;

// LDS of the pruned scan: per wave kPruneWaveBytes, five arrays of SL = 256
// CW corner slots (of which the pruned path uses b3, the exact scan's bound
// per slot, and the first entries of b1 and i1, the waves' minima in that
// scan), the slots of the exact scan, then two counters (exact-scan slots,
// claimed groups); a region of at least `floor` bytes (the IDM lead search
// shares it).
__device__ __forceinline__ ScanLds carve_scan_pruned(void *p, int G, int CW)
{
    float4 *stage = (float4 *)p;
    float *f = (float *)((unsigned char *)p + (size_t)kPruneWaveBytes * G * CW);
    const int SL = 256 * CW;
    int *fl = (int *)(f + 5 * SL);
    return ScanLds{stage, f, f + SL, f + 2 * SL, (int *)(f + 3 * SL), (int *)(f + 4 * SL), fl, fl + SL};
}

__host__ __device__ constexpr size_t scan_pruned_lds_bytes(int G, int CW, size_t floor)
{
    const size_t b = (size_t)kPruneWaveBytes * G * CW + (size_t)256 * CW * 24 + 16;
    return b > floor ? b : align_up(floor, 16);
}

template <int R>
__device__ __forceinline__ void scan_r(const float *stream, int c0, int c1, float4 *stage, const float (&cx)[4],
                                       const float (&cy)[4],
                                       float (&b1)[4], float (&b2)[4], float (&b3)[4], int (&i1)[4], int (&i2)[4])
{
    float x[R], y[R], v1[R], v2[R], v3[R];
    int j1[R], j2[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        x[r] = cx[r]; y[r] = cy[r]; v1[r] = b1[r]; v2[r] = b2[r]; v3[r] = b3[r]; j1[r] = i1[r]; j2[r] = i2[r];
    }
    scan_edges<R>(stream, c0, c1, stage, x, y, v1, v2, v3, j1, j2);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        b1[r] = v1[r]; b2[r] = v2[r]; b3[r] = v3[r]; i1[r] = j1[r]; i2[r] = j2[r];
    }
}

// Off-road scan of the 4*Ns corners of slice objects i0.. against one
// scenario's compacted edges (stream/dir/idx already offset to the scenario,
// E edges, qqmax), then the exact rescan of the candidate chunks (8 lanes per
// corner) that yields the lowest-index nearest point and the signed side of
// every corner.  Waves: w = tid / 64, corner wave cw = w % CW (256 corner
// slots each), edge split g = w / CW (contiguous chunk ranges in index
// order).  Leaves sk[slot] and nidx[slot] (scenario-local point index or -1)
// for slot < 4*Ns.  Contains three block barriers, plus two per corner that
// needs the exact scan of every point (their count is read by every thread
// after a barrier, so the barriers are uniform).
__device__ void offroad_unit(const ObjLds &L, int i0, int Ns, const float *__restrict__ stream,
                             const float2 *__restrict__ edir, const int32_t *__restrict__ eidx, int E, float qqmax,
                             int G, int CW, ScanLds C, float *sk, int *nidx)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
    const int cw = w % CW, g = w / CW;
    const int nslots = 4 * Ns;
    const int SL = 256 * CW;
    const int base = cw * 256;
    const int avail = nslots - base;
    const int Reff = avail <= 0 ? 0 : min(4, (avail + 63) >> 6);
    const int nch = (E + kChunk - 1) / kChunk;
    const int cps = (nch + G - 1) / G;
    const int c0 = min(nch, g * cps), c1 = min(nch, c0 + cps);
    float cx[4], cy[4], b1[4], b2[4], b3[4];
    int i1[4], i2[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        int slot = base + lane + 64 * r;
        slot = min(slot, max(nslots - 1, 0));
        const int o = i0 + (slot >> 2);
        box_corner(L.x[o], L.y[o], L.c[o], L.s[o], 0.5f * L.len[o], 0.5f * L.wid[o], slot & 3, cx[r], cy[r]);
        b1[r] = b2[r] = b3[r] = __builtin_inff();
        i1[r] = i2[r] = -1;
    }
    if (tid == 0)
        *C.nfull = 0;
    float4 *stage = C.stage + (long)w * (kStageBytes / 16);
    if (Reff == 4)
        scan_r<4>(stream, c0, c1, stage, cx, cy, b1, b2, b3, i1, i2);
    else if (Reff == 3)
        scan_r<3>(stream, c0, c1, stage, cx, cy, b1, b2, b3, i1, i2);
    else if (Reff == 2)
        scan_r<2>(stream, c0, c1, stage, cx, cy, b1, b2, b3, i1, i2);
    else if (Reff == 1)
        scan_r<1>(stream, c0, c1, stage, cx, cy, b1, b2, b3, i1, i2);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int slot = base + lane + 64 * r;
        if (r < Reff && slot < nslots) {
            const int at = g * SL + slot;
            C.b1[at] = b1[r];
            C.b2[at] = b2[r];
            C.b3[at] = b3[r];
            C.i1[at] = i1[r];
            C.i2[at] = i2[r];
        }
    }
    __syncthreads();
    for (int slot = tid; slot < nslots; slot += blockDim.x) {
        // best chunk over the splits (ascending splits hold ascending chunks)
        float b = __builtin_inff();
        int bc = -1;
        for (int h = 0; h < G; ++h) {
            const float v = C.b1[h * SL + slot];
            if (v < b) {
                b = v;
                bc = C.i1[h * SL + slot];
            }
        }
        const int o = i0 + (slot >> 2);
        int lo = -1, hi = -1;   // candidate chunks; lo: -1 none, -2 the exact scan of every point
        if (bc >= 0 && L.valid[o]) {
            float x, y;
            box_corner(L.x[o], L.y[o], L.c[o], L.s[o], 0.5f * L.len[o], 0.5f * L.wid[o], slot & 3, x, y);
            const float lim = b + candidate_band(qqmax, x, y);
            int other = -1;        // a second candidate chunk
            bool full = false;     // three or more candidates: exact scan of every chunk
            for (int h = 0; h < G; ++h) {
                const int at = h * SL + slot;
                if (C.b3[at] <= lim)
                    full = true;
                const int cand[2] = {C.i1[at], C.i2[at]};
                const float val[2] = {C.b1[at], C.b2[at]};
                for (int q = 0; q < 2; ++q) {
                    if (val[q] <= lim && cand[q] != bc && cand[q] != other) {
                        if (other < 0)
                            other = cand[q];
                        else
                            full = true;
                    }
                }
            }
            if (full) {
                // rare: left to the whole work-group after the rescans
                C.full[atomicAdd(C.nfull, 1)] = slot;
                lo = -2;
            } else {
                lo = other >= 0 ? min(bc, other) : bc;
                hi = other >= 0 ? max(bc, other) : -1;
            }
        }
        // the candidate chunks wait in the slot's outputs for the rescan
        nidx[slot] = lo;
        sk[slot] = __int_as_float(hi);
    }
    __syncthreads();
    // the exact rescan of the one or two candidate chunks of every corner:
    // kRescanLanes lanes per corner, each 128 / kRescanLanes points of a
    // chunk in ascending order (strict <), then a (D, index) reduction over
    // the corner's lanes that keeps the lowest index of the minimum
    for (int u0 = 0; u0 < nslots * kRescanLanes; u0 += blockDim.x) {   // block-uniform trip count
        const int u = u0 + tid, slot = u / kRescanLanes, rl = u % kRescanLanes;
        const bool act = slot < nslots;
        const int lo = act ? nidx[slot] : -1, hi = act ? __float_as_int(sk[slot]) : -1;
        float best = __builtin_inff(), x = 0.f, y = 0.f;
        int bj = 0x7fffffff;
        if (lo >= 0) {
            const int o = i0 + (slot >> 2);
            box_corner(L.x[o], L.y[o], L.c[o], L.s[o], 0.5f * L.len[o], 0.5f * L.wid[o], slot & 3, x, y);
            rescan_part(stream, lo, rl, E, x, y, best, bj);
            if (hi >= 0)
                rescan_part(stream, hi, rl, E, x, y, best, bj);
        }
        for (int off = kRescanLanes / 2; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off);
            const int oj = __shfl_xor(bj, off);
            if (ob < best || (ob == best && oj < bj)) {
                best = ob;
                bj = oj;
            }
        }
        if (act && rl == 0) {
            // corners for the exact scan of every point keep these defaults
            // until it finds a point
            float s_val = kNoValue;
            int near = -1;
            if (lo >= 0 && bj != 0x7fffffff) {
                const float *ch = stream + kChunkFloats * (bj / kChunk) + (bj % kChunk);
                const float qx = ch[0], qy = ch[kChunk];
                const float2 d = edir[bj];
                s_val = -__builtin_fmaf(d.x, y - qy, -(d.y * (x - qx)));
                near = eidx[bj];
            }
            sk[slot] = s_val;
            nidx[slot] = near;
        }
    }
    __syncthreads();
    // corners with three or more candidate chunks (rare): an exact scan of
    // every edge point by the whole work-group, one corner at a time, with a
    // reduction on (D, index) that keeps the lowest index of the minimum
    const int nf = *C.nfull;
    const int nthr = blockDim.x, nw = nthr >> 6;
    for (int f = 0; f < nf; ++f) {
        const int slot = C.full[f];
        const int o = i0 + (slot >> 2);
        float x, y;
        box_corner(L.x[o], L.y[o], L.c[o], L.s[o], 0.5f * L.len[o], 0.5f * L.wid[o], slot & 3, x, y);
        float best = __builtin_inff();
        int bj = 0x7fffffff;
        // eight points per thread per round, loaded together before use
        for (int j0 = tid; j0 < E; j0 += 8 * nthr) {
            float px[8], py[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = min(j0 + u * nthr, E - 1);
                const float *ch = stream + kChunkFloats * (j / kChunk) + (j % kChunk);
                px[u] = ch[0];
                py[u] = ch[kChunk];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = j0 + u * nthr;
                const float d = edge_d2(px[u], py[u], x, y);
                if (j < E && d < best) {   // j ascends per thread: strict < keeps the lowest
                    best = d;
                    bj = j;
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off);
            const int oj = __shfl_xor(bj, off);
            if (ob < best || (ob == best && oj < bj)) {
                best = ob;
                bj = oj;
            }
        }
        // the merge lists are free after the first barrier: wave results there
        if (lane == 0) {
            C.b1[w] = best;
            C.i1[w] = bj;
        }
        __syncthreads();
        if (tid == 0) {
            float b = __builtin_inff();
            int j = 0x7fffffff;
            for (int v = 0; v < nw; ++v)
                if (C.b1[v] < b || (C.b1[v] == b && C.i1[v] < j)) {
                    b = C.b1[v];
                    j = C.i1[v];
                }
            if (j != 0x7fffffff) {
                const float *ch = stream + kChunkFloats * (j / kChunk) + (j % kChunk);
                const float qx = ch[0], qy = ch[kChunk];
                const float2 d = edir[j];
                sk[slot] = -__builtin_fmaf(d.x, y - qy, -(d.y * (x - qx)));
                nidx[slot] = eidx[j];
            }
        }
        __syncthreads();
    }
}

// The pruned scan of one step for the slice objects i0 .. i0+Ns-1, taken
// in `order` (spatial order, see spatial_order) in groups of GO: the waves
// claim groups from the counter *gctr (zero at entry) until none is left.
// prevq[slot] (slot = 4 il + corner) is the corner's nearest road-edge point
// of the previous step ((+inf, +inf): none), whose distance bounds what the
// scan must look at (scan_group_pruned).  Right after a group's scan its
// wave settles each corner: the best block and a second one within the
// band of it are rescanned exactly (four lanes per corner, the lanes that
// held the corner in the scan), and sk, nidx and prevq of the slot written;
// a corner with three or more blocks within the band is appended to C.full
// with the exact scan's bound in C.b3 (its sk, nidx and prevq are left to
// that scan).  *C.nfull must be zero at entry.
template <int GO>
__device__ void offroad_groups(const ObjLds &L, int i0, int Ns, const float *__restrict__ stream,
                               const float2 *__restrict__ edir, const int32_t *__restrict__ eidx,
                               const float4 *cbox, const float4 *box, int E, float qqmax, const ScanLds &C,
                               const int *order, float2 *prevq, float *sk, int *nidx, int *gctr, ScanCounts &work)
{
    constexpr int CL = 16 / GO;   // lanes per corner
    static_assert(CL == kBlockRescanLanes, "a corner's scan lanes rescan its candidate blocks");
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nch = (E + kChunk - 1) / kChunk;
    const int ngroups = (Ns + GO - 1) / GO;
    float4 *stage = (float4 *)((unsigned char *)C.stage + (long)w * kPruneWaveBytes);
    uint16_t *list = (uint16_t *)(stage + kPruneStageBytes / 16);
    const int k = lane / CL;   // corner of the group: object k / 4, corner k % 4
    for (;;) {
        int gi = 0;
        if (lane == 0)
            gi = atomicAdd(gctr, 1);
        gi = __builtin_amdgcn_readfirstlane(gi);
        if (gi >= ngroups)
            break;
        const int rank = gi * GO + (k >> 2);
        const int il = rank < Ns ? order[rank] : -1;
        const int o = i0 + max(il, 0);
        float cx, cy;
        box_corner(L.x[o], L.y[o], L.c[o], L.s[o], 0.5f * L.len[o], 0.5f * L.wid[o], k & 3, cx, cy);
        float thr = -__builtin_inff();   // needs nothing
        if (il >= 0 && L.valid[o]) {
            const float2 q = prevq[4 * il + (k & 3)];
            thr = edge_d2(q.x, q.y, cx, cy) + 2.0f * candidate_band(qqmax, cx, cy);
        }
        float b1 = __builtin_inff(), b2 = __builtin_inff(), b3 = __builtin_inff();
        int i1 = -1, i2 = -1;
        const float orad = 0.5f * sqrtf(__builtin_fmaf(L.wid[o], L.wid[o], L.len[o] * L.len[o]));
        scan_group_pruned<GO>(stream, cbox, box, nch, stage, list, cx, cy, thr, L.x[o], L.y[o], orad, b1, b2, b3,
                              i1, i2, work);
        // candidate blocks: lo -1 none, -2 the exact scan of every block
        const int part = lane % CL, slot = 4 * il + (k & 3);
        int lo = -1, hi = -1;
        if (il >= 0 && i1 >= 0 && L.valid[o]) {
            const float lim = b1 + candidate_band(qqmax, cx, cy);
            if (b3 <= lim) {
                lo = -2;
                if (part == 0) {
                    C.full[atomicAdd(C.nfull, 1)] = slot;
                    // the exact scan's bound on D (b1 is a minimum of T = D - |c|^2)
                    C.b3[slot] = (b1 + __builtin_fmaf(cy, cy, cx * cx)) + candidate_band(qqmax, cx, cy);
                }
            } else {
                const int other = b2 <= lim && i2 != i1 ? i2 : -1;
                lo = other >= 0 ? min(i1, other) : i1;
                hi = other >= 0 ? max(i1, other) : -1;
            }
        }
        float best = __builtin_inff();
        int bj = 0x7fffffff;
        if (lo >= 0) {
            rescan_block(stream, lo, part, E, cx, cy, best, bj);
            if (hi >= 0)
                rescan_block(stream, hi, part, E, cx, cy, best, bj);
        }
        for (int off = kBlockRescanLanes / 2; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off);
            const int oj = __shfl_xor(bj, off);
            if (ob < best || (ob == best && oj < bj)) {
                best = ob;
                bj = oj;
            }
        }
        if (il >= 0 && part == 0) {
            float s_val = kNoValue;
            int near = -1;
            float2 pq = make_float2(__builtin_inff(), __builtin_inff());
            if (lo >= 0 && bj != 0x7fffffff) {
                const float *ch = stream + kChunkFloats * (bj / kChunk) + (bj % kChunk);
                const float qx = ch[0], qy = ch[kChunk];
                const float2 d = edir[bj];
                s_val = -__builtin_fmaf(d.x, cy - qy, -(d.y * (cx - qx)));
                near = eidx[bj];
                pq = make_float2(qx, qy);
            }
            if (lo != -2)
                prevq[slot] = pq;
            sk[slot] = s_val;
            nidx[slot] = near;
        }
    }
}

// The fused rollout's off-road step for slice objects i0 .. i0+Ns-1 (the
// result of offroad_unit, with the scan pruned: offroad_groups).  prevq
// receives this step's nearest points.  *gctr must be zero at entry; it is
// zero again at return.  *C.nfull must be zero at entry, set so before a
// barrier that precedes the call (the corners of the exact scan are
// counted during the groups); the caller clears it again before the next
// call, after every thread has passed this call.
__device__ void offroad_unit_pruned(const ObjLds &L, int i0, int Ns, const float *__restrict__ stream,
                                    const float2 *__restrict__ edir, const int32_t *__restrict__ eidx,
                                    const float4 *cbox, const float4 *box, int E, float qqmax, ScanLds C, float *sk,
                                    int *nidx, const int *order, float2 *prevq, int *gctr, ScanCounts &work)
{
    const int tid = threadIdx.x, lane = tid & 63;
    offroad_groups<kGroupObjects>(L, i0, Ns, stream, edir, eidx, cbox, box, E, qqmax, C, order, prevq, sk, nidx,
                                  gctr, work);
    __syncthreads();
    if (tid == 0)
        *gctr = 0;
    const int nf = *C.nfull;
    const int nthr = blockDim.x, nw = nthr >> 6, w = tid >> 6;
    for (int f = 0; f < nf; ++f) {
        const int slot = C.full[f];
        const int o = i0 + (slot >> 2);
        float x, y;
        box_corner(L.x[o], L.y[o], L.c[o], L.s[o], 0.5f * L.len[o], 0.5f * L.wid[o], slot & 3, x, y);
        // The exact scan of every block that can hold the nearest point: the
        // point of smallest T (= D - |c|^2 in exact arithmetic) has D within a
        // quarter band of b1 + |c|^2, so the minimum of D is at most that, and
        // a block whose box_lb exceeds lim = b1 + |c|^2 + band (the band also
        // covers the rounding of the sum) holds no point at the minimum.
        const float lim = C.b3[slot];
        float best = __builtin_inff();
        int bj = 0x7fffffff;
        const int nblk = (E + 31) / 32;
        for (int k = tid; k < nblk; k += nthr)
            if (box_lb(box[k], x, y) <= lim)
                for (int q = 0; q < kBlockRescanLanes; ++q)
                    rescan_block(stream, k, q, E, x, y, best, bj);
        for (int off = 32; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off);
            const int oj = __shfl_xor(bj, off);
            if (ob < best || (ob == best && oj < bj)) {
                best = ob;
                bj = oj;
            }
        }
        if (lane == 0) {
            C.b1[w] = best;
            C.i1[w] = bj;
        }
        __syncthreads();
        if (tid == 0) {
            float b = __builtin_inff();
            int j = 0x7fffffff;
            for (int v = 0; v < nw; ++v)
                if (C.b1[v] < b || (C.b1[v] == b && C.i1[v] < j)) {
                    b = C.b1[v];
                    j = C.i1[v];
                }
            float2 pq = make_float2(__builtin_inff(), __builtin_inff());
            if (j != 0x7fffffff) {
                const float *ch = stream + kChunkFloats * (j / kChunk) + (j % kChunk);
                const float qx = ch[0], qy = ch[kChunk];
                const float2 d = edir[j];
                sk[slot] = -__builtin_fmaf(d.x, y - qy, -(d.y * (x - qx)));
                nidx[slot] = eidx[j];
                pq = make_float2(qx, qy);
            }
            prevq[slot] = pq;
        }
        __syncthreads();
    }
}

// A real road-edge point near (x, y), for a pruned scan with no nearest
// point of a previous step: the block whose box has the nearest farthest
// corner (among the chunks whose boxes may hold a point nearer than the best
// chunk's farthest corner; earlier blocks win ties), and in it the nearest
// point of index < E.  Any
// real point bounds the corner's nearest distance (scan_group_pruned); this
// one is close to it.  (+inf, +inf) without edges.
__device__ float2 seed_point(const float *__restrict__ stream, const float4 *cbox, const float4 *box, int E, float x,
                             float y)
{
    const int nch = (E + kChunk - 1) / kChunk;
    auto far_d2 = [&](const float4 b) {   // +inf for an empty box
        const float fx = fabsf(b.x - x) > fabsf(b.y - x) ? b.x : b.y;
        const float fy = fabsf(b.z - y) > fabsf(b.w - y) ? b.z : b.w;
        return edge_d2(fx, fy, x, y);
    };
    // One pass over the chunks, four at a time (their box reads in flight
    // together): fc is the nearest farthest chunk corner so far, and the
    // blocks of every chunk whose box may hold a point nearer than fc are
    // tested.  A chunk tested only because fc was still larger never wins:
    // its blocks' farthest corners lie beyond its nearest point, beyond the
    // final fc, and the best block of the chunk attaining the final fc lies
    // within it.
    float fc = __builtin_inff(), fb = __builtin_inff();
    int bb = -1;
    for (int c0 = 0; c0 < nch; c0 += 4) {
        float4 b[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            b[k] = cbox[min(c0 + k, nch - 1)];   // past the end: the last box again
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            fc = fminf(fc, far_d2(b[k]));
            if (c0 + k < nch && box_lb(b[k], x, y) <= fc) {
                const int c = c0 + k;
                float4 bx[4];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    bx[jj] = box[4 * c + jj];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const float d = far_d2(bx[jj]);
                    if (d < fb) {
                        fb = d;
                        bb = 4 * c + jj;
                    }
                }
            }
        }
    }
    float2 q = make_float2(__builtin_inff(), __builtin_inff());
    if (bb < 0)
        return q;
    // the block's points in ascending order, 16 at a time (four 16-byte
    // loads of x and of y in flight; the chunk's storage covers all 32)
    const float *col = stream + kChunkFloats * (bb >> 2) + 32 * (bb & 3);
    const int n = min(32, E - 32 * bb);
    float best = __builtin_inff();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        float4 X[4], Y[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            X[v] = ((const float4 *)col)[4 * h + v];
            Y[v] = ((const float4 *)(col + kChunk))[4 * h + v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float xs[4] = {X[v].x, X[v].y, X[v].z, X[v].w}, ys[4] = {Y[v].x, Y[v].y, Y[v].z, Y[v].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float d = edge_d2(xs[k], ys[k], x, y);
                if (16 * h + 4 * v + k < n && d < best) {
                    best = d;
                    q = make_float2(xs[k], ys[k]);
                }
            }
        }
    }
    return q;
}

// Spatial order of slice objects i0 .. i0+Ns-1: ascending by the Morton code
// of their 8 m cell (invalid objects last), ties by index, into order[].
// Neighbouring objects then share the groups of the pruned scan.  Two
// barriers.
__device__ __forceinline__ void spatial_order(const ObjLds &L, int i0, int Ns, uint32_t *key, int *order)
{
    for (int il = threadIdx.x; il < Ns; il += blockDim.x) {
        const int o = i0 + il;
        uint32_t k = 0xffffffffu;
        if (L.valid[o]) {
            const uint32_t gx = (uint32_t)min(max((int)floorf(L.x[o] * 0.125f) + 2048, 0), 4095);
            const uint32_t gy = (uint32_t)min(max((int)floorf(L.y[o] * 0.125f) + 2048, 0), 4095);
            k = 0;
            for (int b = 0; b < 12; ++b)
                k |= ((gx >> b) & 1u) << (2 * b) | ((gy >> b) & 1u) << (2 * b + 1);
        }
        key[il] = k;
    }
    __syncthreads();
    // eight lanes per object, each counting the keys j = part (mod 8) below it
    const int part = threadIdx.x & 7;
    for (int il = threadIdx.x >> 3; il < Ns; il += blockDim.x >> 3) {
        const uint32_t k = key[il];
        int rank = 0;
        for (int j = part; j < Ns; j += 8) {
            const uint32_t kj = key[j];
            rank += (kj < k || (kj == k && j < il)) ? 1 : 0;
        }
        rank = lanes_sum8(rank);
        if (part == 0)
            order[rank] = il;
    }
    __syncthreads();
}

__device__ __forceinline__ void load_object(ObjLds &L, int i, const wm_state &st, long g)
{
    L.x[i] = st.x[g];
    L.y[i] = st.y[g];
    L.yaw[i] = st.yaw[g];
    L.vx[i] = st.vx[g];
    L.vy[i] = st.vy[g];
    L.len[i] = st.length[g];
    L.wid[i] = st.width[g];
    L.valid[i] = st.valid[g];
    float s, c;
    sincosf(L.yaw[i], &s, &c);
    L.c[i] = c;
    L.s[i] = s;
}

__device__ __forceinline__ void store_object(const ObjLds &L, int i, const wm_state &st, long g)
{
    st.x[g] = L.x[i];
    st.y[g] = L.y[i];
    st.yaw[g] = L.yaw[i];
    st.vx[g] = L.vx[i];
    st.vy[g] = L.vy[i];
    st.length[g] = L.len[i];
    st.width[g] = L.wid[i];
    st.valid[g] = L.valid[i];
}

// Carve the LDS object arrays for up to maxN objects out of `p`; returns the
// first byte after them.
__device__ __forceinline__ unsigned char *carve_objects(unsigned char *p, int maxN, ObjLds &L)
{
    float *f = (float *)p;
    L.x = f;
    L.y = f + maxN;
    L.yaw = f + 2 * maxN;
    L.vx = f + 3 * maxN;
    L.vy = f + 4 * maxN;
    L.len = f + 5 * maxN;
    L.wid = f + 6 * maxN;
    L.c = f + 7 * maxN;
    L.s = f + 8 * maxN;
    uint8_t *b = (uint8_t *)(f + 9 * maxN);
    L.valid = b;
    L.ctrl = b + maxN;
    L.infeas = b + 2 * maxN;
    return p + align_up((size_t)maxN * 39, 16);
}

// ---------------------------------------------------------------------------
// Plain kernels (one launch per operation and step).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dynamics(StepArgs A)
{
    const int s = blockIdx.x;
    const int o0 = A.obj_off[s], o1 = A.obj_off[s + 1];
    for (int g = o0 + (int)threadIdx.x; g < o1; g += blockDim.x) {
        const bool ctrl = A.act.controlled[g];
        float x, y, yaw, vx, vy, len, wid;
        uint8_t valid;
        if (!ctrl) {
            x = A.log_next.x[g]; y = A.log_next.y[g]; yaw = A.log_next.yaw[g];
            vx = A.log_next.vx[g]; vy = A.log_next.vy[g]; len = A.log_next.length[g];
            wid = A.log_next.width[g]; valid = A.log_next.valid[g];
        } else {
            x = A.cur.x[g]; y = A.cur.y[g]; yaw = A.cur.yaw[g]; vx = A.cur.vx[g]; vy = A.cur.vy[g];
            len = A.cur.length[g]; wid = A.cur.width[g]; valid = A.cur.valid[g];
            if (valid)
                bicycle_forward(x, y, yaw, vx, vy, A.act.accel[g], A.act.curvature[g], A.dt);
        }
        A.next.x[g] = x; A.next.y[g] = y; A.next.yaw[g] = yaw; A.next.vx[g] = vx; A.next.vy[g] = vy;
        A.next.length[g] = len; A.next.width[g] = wid; A.next.valid[g] = valid;
        if (A.log_div) {
            float d = 0.f;
            if (valid && A.log_next.valid[g]) {
                const float dx = x - A.log_next.x[g], dy = y - A.log_next.y[g];
                d = sqrtf(__builtin_fmaf(dy, dy, dx * dx));
            }
            A.log_div[g] = d;
        }
        if (A.infeasible) {
            const bool both = valid && A.cur.valid[g];
            A.infeasible[g] = both ? infeasible_transition(A.cur.vx[g], A.cur.vy[g], A.cur.yaw[g], vx, vy, A.dt) : 0;
        }
    }
}

// Sparse reward of Sec. 5.2 from the step's masks: -1[collision] - 1[off-road].
// One block per scenario (so one-scenario views of a batch stay in range).
__global__ __launch_bounds__(256) void k_reward(const int32_t *__restrict__ obj_off, const uint8_t *__restrict__ col,
                                                const uint8_t *__restrict__ off, float *__restrict__ reward)
{
    const int s = blockIdx.x;
    for (int g = obj_off[s] + (int)threadIdx.x; g < obj_off[s + 1]; g += blockDim.x)
        reward[g] = -(float)col[g] - (off ? (float)off[g] : 0.f);
}

__global__ __launch_bounds__(256) void k_inverse(int n, wm_state cur, wm_state nxt, float dt, float *__restrict__ accel,
                                                 float *__restrict__ curv, uint8_t *__restrict__ vout)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n)
        return;
    const bool ok = cur.valid[g] && nxt.valid[g];
    float a = 0.f, k = 0.f;
    if (ok)
        inverse_kinematics(cur.vx[g], cur.vy[g], cur.yaw[g], nxt.vx[g], nxt.vy[g], dt, a, k);
    accel[g] = a;
    curv[g] = k;
    if (vout)
        vout[g] = (uint8_t)ok;
}

// Plain collision metric: block (scenario s, slice blockIdx.y) of U objects.
__global__ __launch_bounds__(256) void k_overlap(OverlapArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    ObjLds L;
    float *red = (float *)carve_objects(smem, A.maxN, L);
    const int s = blockIdx.x;
    const int o0 = A.obj_off[s], N = A.obj_off[s + 1] - o0;
    const int i0 = blockIdx.y * A.U;
    if (i0 >= N)
        return;
    const int Ns = min(A.U, N - i0);
    for (int i = threadIdx.x; i < N; i += blockDim.x)
        load_object(L, i, A.st, o0 + i);
    __syncthreads();
    const int P = blockDim.x / A.U;
    float *rm = A.margin ? A.margin + A.pair_off[s] + (long)i0 * N : nullptr;
    uint8_t *rk = A.mask ? A.mask + A.pair_off[s] + (long)i0 * N : nullptr;
    overlap_partial(L, N, i0, Ns, A.U, P, red, nullptr, rm, rk);
    __syncthreads();
    for (int il = threadIdx.x; il < Ns; il += blockDim.x) {
        float m = kNoValue;
        for (int p = 0; p < P; ++p)
            m = fmaxf(m, red[p * A.U + il]);
        const long g = o0 + i0 + il;
        if (A.collision)
            A.collision[g] = (uint8_t)(m > 0.f);
        if (A.max_margin)
            A.max_margin[g] = m;
    }
}

// Plain off-road metric: block (scenario s, slice blockIdx.y) of 64*CW objects.
__global__ __launch_bounds__(1024) void k_offroad(OffroadArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    ObjLds L;
    unsigned char *p = carve_objects(smem, 64 * A.CW, L);
    const int SL = 256 * A.CW;
    const ScanLds C = carve_scan(p, A.G, SL);
    float *sk = (float *)(p + scan_lds_bytes(A.G, A.CW));
    int *nidx = (int *)(sk + SL);
    const int s = blockIdx.x;
    const int o0 = __builtin_amdgcn_readfirstlane(A.obj_off[s]);
    const int N = __builtin_amdgcn_readfirstlane(A.obj_off[s + 1]) - o0;
    const int U = 64 * A.CW;
    const int i0 = blockIdx.y * U;
    if (i0 >= N)
        return;
    const int Ns = min(U, N - i0);
    for (int i = threadIdx.x; i < Ns; i += blockDim.x)
        load_object(L, i, A.st, o0 + i0 + i);
    __syncthreads();
    const long eb = edge_base(__builtin_amdgcn_readfirstlane(A.rg_off[s]), s);
    // the count comes from the workspace: clamped to the scenario's capacity
    // so that a stale workspace can only give wrong values, never an access
    // outside the scenario's edge slots
    const int E = __builtin_amdgcn_readfirstlane(
        max(0, min(A.E.count[s], A.rg_off[s + 1] - A.rg_off[s])));
    const float qqmax = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(A.E.qqmax[s])));
    offroad_unit(L, 0, Ns, A.E.stream + 3 * eb, A.E.dir + eb, A.E.idx + eb, E, qqmax, A.G, A.CW, C, sk, nidx);
    for (int il = threadIdx.x; il < Ns; il += blockDim.x) {
        float m = kNoValue;
        for (int k = 0; k < 4; ++k)
            m = fmaxf(m, sk[4 * il + k]);
        const long g = o0 + i0 + il;
        if (A.offroad)
            A.offroad[g] = (uint8_t)(m > 0.f);
        if (A.margin)
            A.margin[g] = m;
        if (A.nearest)
            for (int k = 0; k < 4; ++k)
                A.nearest[4 * g + k] = nidx[4 * il + k];
    }
}

// ---------------------------------------------------------------------------
// Persistent fused rollout.  Each work-group repeatedly takes the next unit
// (scenario s, slice) from the queue and runs all T steps for it: dynamics of
// all N_s objects (needed by the slice's pairs), then for the slice objects
// the overlap, off-road, log divergence, loss terms, outputs and checkpoints.
// ---------------------------------------------------------------------------
// Largest scenario for which the IDM lead search keeps a per-agent bit mask
// of candidate objects in LDS (maxN^2 / 8 bytes); larger ones test every
// object.
constexpr int kIdmMaskMaxN = 256;

// Per-wave LDS scratch of the lead search (floats): poses x, y, yaw of up
// to WM_MAX_IDM_POSES lookahead poses, then the candidate list (ints).
constexpr int kIdmPoseScratch = 3 * 64;
static_assert(WM_MAX_IDM_POSES <= 64, "one lane per lookahead pose");

// The fused rollout's scan region in LDS: the pruned scan's, at least as
// large as the lead search's per-wave scratch (poses and a candidate list of
// maxN) for every wave.
__host__ __device__ constexpr size_t rollout_scan_bytes(int G, int CW, int maxN)
{
    return scan_pruned_lds_bytes(G, CW, (size_t)G * CW * (kIdmPoseScratch + maxN) * 4);
}

__device__ __forceinline__ int wave_min(int v)
{
    for (int d = 32; d > 0; d >>= 1)
        v = min(v, __shfl_xor(v, d));
    return v;
}

// IDM sim agents, per step from the states at t-1 in LDS: the lead of every
// agent (the first lookahead pose, then the lowest object index, whose box
// overlaps another valid object's current box), then each agent's
// acceleration into ia[].  All poses of agent i lie within M * step (arc
// length) of its pose at sig[i], so only objects within M * step + r_i + r_j
// of that point (r: half diagonal) can overlap one of them; with maxN <=
// kIdmMaskMaxN those candidates are collected first as a bit mask per agent,
// one 32-bit word per half-wave ballot.  Then one wave per agent: lane m
// computes lookahead pose m + 1, the candidates are listed in ascending
// index order, and the (pose, candidate) pairs are tested 64 at a time in
// pose-major order, so the first pass with an overlap holds the lead (a
// wave minimum of pose * 2048 + index).  wscr: the off-road scratch, unused
// at this point of the step.  Contains three block barriers.
__device__ __forceinline__ void idm_leads(const RollArgs &A, const ObjLds &L, int o0, int N, const float *sig, float *ia,
                                          int *lk, const uint8_t *agent, float *pc, uint32_t *mask, float *wscr)
{
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6, nw = nthr >> 6;
    const int M = A.idm.lookahead_poses;
    const bool use_mask = A.maxN <= kIdmMaskMaxN;
    const int W = (N + 31) >> 5;
    float *rad = ia;   // circumradius per object, until the accelerations are written
    // (pc holds each agent's pose at sig, kept by idm_move)
    for (int i = tid; i < N; i += nthr)
        rad[i] = 0.5f * sqrtf(__builtin_fmaf(L.wid[i], L.wid[i], L.len[i] * L.len[i]));
    __syncthreads();
    const float reach = (float)M * A.idm.lookahead_step;
    if (use_mask) {
        // word q = (agent i, objects 32 w .. 32 w + 31): lane b of a half-wave
        // tests object 32 w + b, and the half-wave's ballot is the word
        const int half = lane >> 5, bit = lane & 31;
        for (int q = 2 * wv + half; q < N * W; q += 2 * nw) {
            const int i = q / W, j = 32 * (q - i * W) + bit;
            bool hit = false;
            if (agent[i] && j < N && j != i && L.valid[j]) {
                const float dx = L.x[j] - pc[2 * i], dy = L.y[j] - pc[2 * i + 1];
                const float rr = reach + rad[i] + rad[j] + 1e-2f;
                hit = __builtin_fmaf(dy, dy, dx * dx) <= rr * rr;
            }
            const uint64_t b = __ballot(hit);
            if (bit == 0)
                mask[q] = (uint32_t)(b >> (32 * half));
        }
        __syncthreads();
    }
    // a wave's share of the scratch: poses, candidate list, then (when it
    // fits) the agent's path arc lengths for an LDS search
    const int per_wave = (int)(rollout_scan_bytes(A.G, A.CW, A.maxN) / 4 / nw);
    float *px = wscr + (size_t)wv * per_wave, *py = px + 64, *pyw = px + 128;
    int *cl = (int *)(px + kIdmPoseScratch);
    float *wcol = px + kIdmPoseScratch + A.maxN;
    const bool col_lds = kIdmPoseScratch + A.maxN + A.T + 1 <= per_wave;
    const float step = A.idm.lookahead_step;
    for (int i = wv; i < N; i += nw) {   // one agent per wave (uniform)
        if (!agent[i])
            continue;
        const float4 *path = A.idmP + (long)(o0 + i) * (A.T + 1);
        if (col_lds) {
            for (int k = lane; k <= A.T; k += 64)
                wcol[k] = path[k].w;
            __builtin_amdgcn_wave_barrier();
        }
        // lookahead pose m = lane + 1, if it lies on the path
        const int m = lane + 1;
        const float sm = __builtin_fmaf((float)m, step, sig[i]);
        const bool live = m <= M && sm <= path[A.T].w;
        float x = 0.f, y = 0.f, yaw = 0.f;
        if (live) {
            const int lo = col_lds ? idm_segment([&](int k) { return wcol[k]; }, A.T, sm)
                                   : idm_segment([&](int k) { return path[k].w; }, A.T, sm);
            idm_interp(path, A.T, lo, sm, x, y, yaw);
        }
        px[lane] = x;
        py[lane] = y;
        pyw[lane] = yaw;
        const int nlive = __popcll(__ballot(live));   // poses 1..nlive (arc length grows with m)
        // candidates in ascending index order
        int nc = 0;
        for (int w0 = 0; w0 < W; w0 += 2) {
            const int w = w0 + (lane >> 5), j = 32 * w + (lane & 31);
            bool c = false;
            if (w < W && j < N && j != i && L.valid[j])
                c = use_mask ? ((mask[i * W + w] >> (lane & 31)) & 1u) != 0u : true;
            const uint64_t bal = __ballot(c);
            if (c)
                cl[nc + __popcll(bal & ((1ull << lane) - 1ull))] = j;
            nc += __popcll(bal);
        }
        __builtin_amdgcn_wave_barrier();   // the wave's LDS writes above precede its reads below
        const int npair = nlive * nc;
        const float rinv = 1.0f / (float)max(nc, 1);
        const float ra = rad[i];
        int lead = 0x7fffffff;
        for (int p0 = 0; p0 < npair; p0 += 64) {
            const int pr = p0 + lane;
            int key = 0x7fffffff;
            if (pr < npair) {
                int mi = (int)(((float)pr + 0.5f) * rinv), q = pr - mi * nc;   // pose index, candidate slot
                if (q < 0) {
                    --mi;
                    q += nc;
                } else if (q >= nc) {
                    ++mi;
                    q -= nc;
                }
                const int j = cl[q];
                const float ax = px[mi], ay = py[mi];
                // boxes lie within their circumscribed circles
                const float dx = L.x[j] - ax, dy = L.y[j] - ay;
                const float rr = ra + rad[j] + 1e-3f;
                if (__builtin_fmaf(dy, dy, dx * dx) <= rr * rr) {
                    float ps, pcs;
                    sincosf(pyw[mi], &ps, &pcs);
                    const Box a{ax, ay, pcs, ps, 0.5f * L.len[i], 0.5f * L.wid[i]};
                    const Box b{L.x[j], L.y[j], L.c[j], L.s[j], 0.5f * L.len[j], 0.5f * L.wid[j]};
                    if (sat_margin(a, b) > 0.f)
                        key = (mi + 1) * 2048 + j;
                }
            }
            if (__ballot(key != 0x7fffffff)) {   // later passes hold only later poses
                lead = wave_min(key);
                break;
            }
        }
        if (lane == 0)
            lk[i] = lead;
        __builtin_amdgcn_wave_barrier();   // reads of this agent's scratch precede the next agent's writes
    }
    __syncthreads();
    for (int i = tid; i < N; i += nthr) {
        if (!agent[i])
            continue;
        const int key = lk[i];
        const float v = sqrtf(__builtin_fmaf(L.vy[i], L.vy[i], L.vx[i] * L.vx[i]));
        if (key == 0x7fffffff) {
            ia[i] = idm_accel(A.idm, v, false, 0.f, 0.f);
        } else {
            const int m = key >> 11, j = key & 2047;
            const float vl = __builtin_fmaf(L.vy[j], L.s[i], L.vx[j] * L.c[i]);
            ia[i] = idm_accel(A.idm, v, true, (float)(m - 1) * A.idm.lookahead_step, vl);
        }
    }
    __syncthreads();
}

// Advance IDM agent i (global g) with acceleration a along its path; the
// next state's length, width and valid come from log row `row`.  sg[i] is
// the path segment of sig[i] (progress never decreases, so the new segment
// is searched from it); pc receives the new pose's position.
__device__ __forceinline__ void idm_move(const RollArgs &A, const ObjLds &L, int i, long g, long row, float *sig,
                                         int *sg, float *pc, float a)
{
    const float dt = A.dt;
    const float v = sqrtf(__builtin_fmaf(L.vy[i], L.vy[i], L.vx[i] * L.vx[i]));
    float vn = __builtin_fmaf(a, dt, v), adv;
    if (vn >= 0.f) {
        adv = __builtin_fmaf(v, dt, 0.5f * a * dt * dt);
    } else {
        adv = v * v / (2.0f * -a);
        vn = 0.f;
    }
    const float4 *path = A.idmP + g * (A.T + 1);
    const float Lend = path[A.T].w;
    if (sig[i] + adv >= Lend) {   // the end of the path: halt there
        sig[i] = Lend;
        vn = 0.f;
    } else {
        sig[i] += adv;
    }
    float x, y, yaw, sn, cs;
    const int lo = idm_segment_from(path, A.T, sig[i], sg[i]);
    sg[i] = lo;
    idm_interp(path, A.T, lo, sig[i], x, y, yaw);
    pc[2 * i] = x;
    pc[2 * i + 1] = y;
    sincosf(yaw, &sn, &cs);
    L.x[i] = x;
    L.y[i] = y;
    L.yaw[i] = yaw;
    L.vx[i] = vn * cs;
    L.vy[i] = vn * sn;
    L.c[i] = cs;
    L.s[i] = sn;
    L.len[i] = A.log.length[row + g];
    L.wid[i] = A.log.width[row + g];
    L.valid[i] = A.log.valid[row + g];
}

// The logged path of every object, rows 0..T, object-major as (x, y, yaw,
// cumulative arc length), and the IDM agent flag: uncontrolled and valid in
// every row.
__global__ __launch_bounds__(256) void k_idm_paths(int n, int T, wm_state log, const uint8_t *__restrict__ controlled,
                                                   float4 *__restrict__ path, uint8_t *__restrict__ agent)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n)
        return;
    float4 *p = path + (long)g * (T + 1);
    bool ok = !controlled[g] && log.valid[g];
    float acc = 0.f;
    p[0] = make_float4(log.x[g], log.y[g], log.yaw[g], 0.f);
    for (int k = 1; k <= T; ++k) {
        const long a = (long)(k - 1) * n + g, b = (long)k * n + g;
        const float dx = log.x[b] - log.x[a], dy = log.y[b] - log.y[a];
        acc = acc + sqrtf(__builtin_fmaf(dy, dy, dx * dx));
        p[k] = make_float4(log.x[b], log.y[b], log.yaw[b], acc);
        ok = ok && log.valid[b];
    }
    agent[g] = (uint8_t)ok;
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_rollout(RollArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    ObjLds L;
    unsigned char *p = carve_objects(smem, A.maxN, L);
    const int U = 64 * A.CW;
    const int SL = 256 * A.CW;
    const int nthr = blockDim.x;
    const int P = nthr / U;
    const ScanLds C = carve_scan_pruned(p, A.G, A.CW);
    float *sk = (float *)(p + rollout_scan_bytes(A.G, A.CW, A.maxN));
    int *nidx = (int *)(sk + SL);
    float *red = (float *)(nidx + SL);
    float *wsum = red + nthr;
    float *sig = wsum + 16;              // IDM: path progress
    float *ia = sig + A.maxN;            // IDM: acceleration of the step
    int *lk = (int *)(ia + A.maxN);      // IDM: lead key m * 2048 + j
    uint8_t *agent = (uint8_t *)(lk + A.maxN);
    float *pc = (float *)(agent + align_up((size_t)A.maxN, 16));   // IDM: pose at sig (x, y)
    int *sg = (int *)(pc + 2 * A.maxN);                               // IDM: path segment of sig
    uint32_t *mask = (uint32_t *)(sg + A.maxN);                       // IDM: candidate bit masks
    // the pruned off-road scan: the scenario's chunk and block boxes (when at
    // most kLdsBoxChunks chunks), each corner's nearest road-edge point of the
    // previous step, spatial keys and order of the slice's objects, the
    // group counter
    float4 *lcbox = (float4 *)align_up((size_t)(mask + (A.maxN <= kIdmMaskMaxN ? A.maxN * ((A.maxN + 31) / 32) : 0)), 16);
    float4 *lbox = lcbox + kLdsBoxChunks;
    float2 *prevq = (float2 *)(lbox + 4 * kLdsBoxChunks);
    uint32_t *okey = (uint32_t *)(prevq + 4 * U);
    int *order = (int *)(okey + U);
    int *gctr = order + U;
    // the objects' boxes packed for the overlap (at most kPackedMaxN objects)
    const bool packed = A.maxN <= kPackedMaxN;
    float4 *obox = (float4 *)align_up((size_t)(gctr + 1), 16);
    __shared__ int s_unit;
    const int tid = threadIdx.x;
    const long n = A.n;
    ScanCounts work{0u, 0u, 0u};
    for (;;) {
        if (tid == 0)
            s_unit = atomicAdd(A.counter, 1);
        __syncthreads();
        // the unit, its scenario and the scan's chunk ranges are made provably
        // wave-uniform (scalar registers)
        const int q = __builtin_amdgcn_readfirstlane(s_unit);
        if (q >= __builtin_amdgcn_readfirstlane(A.counter[1])) {
            // this wave's work counts (kRollCounts after the queue counters)
            if ((tid & 63) == 0) {
                unsigned long long *wc = (unsigned long long *)(A.counter + kRollCounts);
                atomicAdd(wc, (unsigned long long)work.folded);
                atomicAdd(wc + 1, (unsigned long long)work.chunk_tests);
                atomicAdd(wc + 2, (unsigned long long)work.block_tests);
            }
            break;
        }
        const int2 un = A.units[q];
        const int s = __builtin_amdgcn_readfirstlane(un.x), slice = __builtin_amdgcn_readfirstlane(un.y);
        const int o0 = __builtin_amdgcn_readfirstlane(A.obj_off[s]);
        const int N = __builtin_amdgcn_readfirstlane(A.obj_off[s + 1]) - o0;
        const int i0 = slice * U, Ns = min(U, N - i0);
        const long eb = A.has_rg ? edge_base(__builtin_amdgcn_readfirstlane(A.rg_off[s]), s) : 0;
        const int E = A.has_rg ? __builtin_amdgcn_readfirstlane(
                                     max(0, min(A.E.count[s], A.rg_off[s + 1] - A.rg_off[s])))
                               : 0;
        const float qqmax = A.has_rg ? __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(A.E.qqmax[s]))) : 0.f;
        for (int i = tid; i < N; i += nthr) {
            load_object(L, i, A.init, o0 + i);
            L.ctrl[i] = A.act.controlled[o0 + i];
            if (A.has_idm) {
                sig[i] = 0.f;
                agent[i] = A.idmA[o0 + i];
                if (agent[i]) {   // the pose at progress 0 and its segment
                    const float4 *path = A.idmP + (long)(o0 + i) * (A.T + 1);
                    const int lo = idm_segment([&](int k) { return path[k].w; }, A.T, 0.f);
                    float x, y, yaw;
                    idm_interp(path, A.T, lo, 0.f, x, y, yaw);
                    sg[i] = lo;
                    pc[2 * i] = x;
                    pc[2 * i + 1] = y;
                }
            }
        }
        if (A.has_ckpt)
            for (int il = tid; il < Ns; il += nthr)
                store_object(L, i0 + il, A.ckpt, o0 + i0 + il);
        for (int k = tid; k < 4 * U; k += nthr)
            prevq[k] = make_float2(__builtin_inff(), __builtin_inff());
        const int nch = (E + kChunk - 1) / kChunk;
        const bool lds_boxes = nch <= kLdsBoxChunks;
        if (lds_boxes) {
            for (int k = tid; k < nch; k += nthr)
                lcbox[k] = A.E.cbox[eb / kChunk + k];
            for (int k = tid; k < 4 * nch; k += nthr)
                lbox[k] = A.E.box[eb / kBoxPts + k];
        }
        if (tid == 0)
            *gctr = 0;
        __syncthreads();
        if (A.has_rg) {
            // the first step's bounds: real points near the initial corners
            for (int slot = tid; slot < 4 * Ns; slot += nthr) {
                const int o = i0 + (slot >> 2);
                float x, y;
                box_corner(L.x[o], L.y[o], L.c[o], L.s[o], 0.5f * L.len[o], 0.5f * L.wid[o], slot & 3, x, y);
                prevq[slot] = seed_point(A.E.stream + 3 * eb, lds_boxes ? lcbox : A.E.cbox + eb / kChunk,
                                         lds_boxes ? lbox : A.E.box + eb / kBoxPts, E, x, y);
            }
            __syncthreads();
        }
        float my_loss = 0.f;
        for (int t = 1; t <= A.T; ++t) {
            const long row = (long)t * n, arow = (long)(t - 1) * n;
            if (A.has_idm)
                idm_leads(A, L, o0, N, sig, ia, lk, agent, pc, mask, (float *)C.stage);
            for (int i = tid; i < N; i += nthr) {
                const long g = o0 + i;
                const float pvx = L.vx[i], pvy = L.vy[i], pyaw = L.yaw[i];
                const bool pvalid = L.valid[i];
                if (!L.ctrl[i] && A.has_idm && agent[i]) {
                    idm_move(A, L, i, g, row, sig, sg, pc, ia[i]);
                } else if (!L.ctrl[i]) {
                    load_object(L, i, A.log, row + g);
                } else if (L.valid[i]) {
                    float x = L.x[i], y = L.y[i], yaw = L.yaw[i], vx = L.vx[i], vy = L.vy[i];
                    bicycle_forward(x, y, yaw, vx, vy, A.act.accel[arow + g], A.act.curvature[arow + g], A.dt);
                    L.x[i] = x; L.y[i] = y; L.yaw[i] = yaw; L.vx[i] = vx; L.vy[i] = vy;
                    float sn, cs;
                    sincosf(yaw, &sn, &cs);
                    L.c[i] = cs;
                    L.s[i] = sn;
                }
                L.infeas[i] = (pvalid && L.valid[i]) ? infeasible_transition(pvx, pvy, pyaw, L.vx[i], L.vy[i], A.dt)
                                                    : (uint8_t)0;
                if (packed) {
                    obox[2 * i] = make_float4(L.x[i], L.y[i], L.c[i], L.s[i]);
                    obox[2 * i + 1] = make_float4(0.5f * L.len[i], 0.5f * L.wid[i], L.valid[i] ? 1.f : 0.f, 0.f);
                }
            }
            __syncthreads();
            for (int il = tid; il < Ns; il += nthr) {
                const int i = i0 + il;
                const long g = o0 + i;
                if (A.met.infeasible)
                    A.met.infeasible[arow + g] = L.infeas[i];
                if (A.has_traj)
                    store_object(L, i, A.traj, arow + g);
                if (A.has_ckpt && t % A.ckpt_every == 0 && t < A.T)
                    store_object(L, i, A.ckpt, (long)(t / A.ckpt_every) * n + g);
                const bool both = L.valid[i] && A.log.valid[row + g];
                const float dx = L.x[i] - A.log.x[row + g], dy = L.y[i] - A.log.y[row + g];
                const float d2 = __builtin_fmaf(dy, dy, dx * dx);
                if (A.met.log_div)
                    A.met.log_div[arow + g] = both ? sqrtf(d2) : 0.f;
                if (A.want_loss && both && L.ctrl[i])
                    my_loss += d2;
            }
            if (packed)
                overlap_partial_packed(L, obox, N, i0, Ns, U, P, red, A.want_loss ? &my_loss : nullptr);
            else
                overlap_partial(L, N, i0, Ns, U, P, red, A.want_loss ? &my_loss : nullptr, nullptr, nullptr);
            if (A.has_rg) {
                if (tid == 0)
                    *C.nfull = 0;   // every thread has read the last step's count (barriers since)
                // objects move little in a step: the spatial order is renewed
                // every kReorderSteps steps (it only shapes the groups; every
                // corner's result is exact whatever the groups)
                if ((t - 1) % kReorderSteps == 0)
                    spatial_order(L, i0, Ns, okey, order);
                else
                    __syncthreads();
                offroad_unit_pruned(L, i0, Ns, A.E.stream + 3 * eb, A.E.dir + eb, A.E.idx + eb,
                                    lds_boxes ? lcbox : A.E.cbox + eb / kChunk,
                                    lds_boxes ? lbox : A.E.box + eb / kBoxPts, E, qqmax, C, sk, nidx, order, prevq,
                                    gctr, work);
            } else {
                __syncthreads();
            }
            for (int il = tid; il < Ns; il += nthr) {
                float m = kNoValue;
                for (int pp = 0; pp < P; ++pp)
                    m = fmaxf(m, red[pp * U + il]);
                const long g = arow + o0 + i0 + il;
                if (A.met.collision)
                    A.met.collision[g] = (uint8_t)(m > 0.f);
                if (A.met.overlap_margin)
                    A.met.overlap_margin[g] = m;
                float r = kNoValue;
                if (A.has_rg) {
                    for (int k = 0; k < 4; ++k)
                        r = fmaxf(r, sk[4 * il + k]);
                    if (A.met.offroad)
                        A.met.offroad[g] = (uint8_t)(r > 0.f);
                    if (A.met.offroad_margin)
                        A.met.offroad_margin[g] = r;
                }
                if (A.met.reward)
                    A.met.reward[g] = -(float)(m > 0.f) - (float)(r > 0.f);
            }
            __syncthreads();
        }
        if (A.want_loss) {
            // deterministic block sum: wave reduction then fixed-order sum
            float v = my_loss;
            for (int off = 32; off > 0; off >>= 1)
                v += __shfl_xor(v, off);
            if ((tid & 63) == 0)
                wsum[tid >> 6] = v;
            __syncthreads();
            if (tid == 0) {
                float tot = 0.f;
                for (int w = 0; w < nthr / 64; ++w)
                    tot += wsum[w];
                A.lossp[A.uoff[s] + slice] = tot;
            }
        }
        __syncthreads();
    }
}

// The per-step off-road metric with the fused rollout's pruned scan (for
// tunings of at most 512 threads): one work-group per (scenario, slice of 64
// CW objects), each corner's scan bounded by a real point near it
// (seed_point) instead of a previous step's nearest point.
__global__ __launch_bounds__(512) void k_offroad_pruned(OffroadArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    ObjLds L;
    const int U = 64 * A.CW, SL = 256 * A.CW, nthr = blockDim.x;
    unsigned char *p = carve_objects(smem, U, L);
    const ScanLds C = carve_scan_pruned(p, A.G, A.CW);
    float *sk = (float *)(p + scan_pruned_lds_bytes(A.G, A.CW, 0));
    int *nidx = (int *)(sk + SL);
    float4 *lcbox = (float4 *)(nidx + SL);
    float4 *lbox = lcbox + kLdsBoxChunks;
    float2 *prevq = (float2 *)(lbox + 4 * kLdsBoxChunks);
    uint32_t *okey = (uint32_t *)(prevq + 4 * U);
    int *order = (int *)(okey + U);
    int *gctr = order + U;
    const int s = blockIdx.x, tid = threadIdx.x;
    const int o0 = __builtin_amdgcn_readfirstlane(A.obj_off[s]);
    const int N = __builtin_amdgcn_readfirstlane(A.obj_off[s + 1]) - o0;
    const int i0 = blockIdx.y * U;
    if (i0 >= N)
        return;
    const int Ns = min(U, N - i0);
    const long eb = edge_base(__builtin_amdgcn_readfirstlane(A.rg_off[s]), s);
    // the count comes from the workspace, clamped to the scenario's capacity
    const int E = __builtin_amdgcn_readfirstlane(max(0, min(A.E.count[s], A.rg_off[s + 1] - A.rg_off[s])));
    const float qqmax = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(A.E.qqmax[s])));
    const int nch = (E + kChunk - 1) / kChunk;
    const bool lds_boxes = nch <= kLdsBoxChunks;
    const float4 *gcbox = A.E.cbox + eb / kChunk, *gbox = A.E.box + eb / kBoxPts;
    for (int i = tid; i < Ns; i += nthr)
        load_object(L, i, A.st, o0 + i0 + i);
    if (lds_boxes) {
        for (int k = tid; k < nch; k += nthr)
            lcbox[k] = gcbox[k];
        for (int k = tid; k < 4 * nch; k += nthr)
            lbox[k] = gbox[k];
    }
    if (tid == 0) {
        *gctr = 0;
        *C.nfull = 0;
    }
    __syncthreads();
    const float4 *cbox = lds_boxes ? lcbox : gcbox, *box = lds_boxes ? lbox : gbox;
    // each corner's bound: a real point near it
    for (int slot = tid; slot < 4 * Ns; slot += nthr) {
        const int o = slot >> 2;
        float x, y;
        box_corner(L.x[o], L.y[o], L.c[o], L.s[o], 0.5f * L.len[o], 0.5f * L.wid[o], slot & 3, x, y);
        prevq[slot] = seed_point(A.E.stream + 3 * eb, cbox, box, E, x, y);
    }
    spatial_order(L, 0, Ns, okey, order);   // its first barrier orders prevq too
    ScanCounts work{0u, 0u, 0u};
    offroad_unit_pruned(L, 0, Ns, A.E.stream + 3 * eb, A.E.dir + eb, A.E.idx + eb, cbox, box, E, qqmax, C, sk,
                        nidx, order, prevq, gctr, work);
    __syncthreads();
    for (int il = tid; il < Ns; il += nthr) {
        float m = kNoValue;
        for (int k = 0; k < 4; ++k)
            m = fmaxf(m, sk[4 * il + k]);
        const long g = o0 + i0 + il;
        if (A.offroad)
            A.offroad[g] = (uint8_t)(m > 0.f);
        if (A.margin)
            A.margin[g] = m;
        if (A.nearest)
            for (int k = 0; k < 4; ++k)
                A.nearest[4 * g + k] = nidx[4 * il + k];
    }
}

__global__ void k_loss_reduce(int S, const int32_t *__restrict__ uoff, const float *__restrict__ lossp,
                              float *__restrict__ loss)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    float tot = 0.f;
    for (int u = uoff[s]; u < uoff[s + 1]; ++u)
        tot += lossp[u];
    loss[s] = tot;
}

} // namespace wm

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace wm {

static size_t objects_lds(int maxN) { return align_up((size_t)maxN * 39, 16); }

void launch_compact_edges(const wm_batch &b, const wm_roadgraph &rg, unsigned char *ws, const WsLayout &L,
                          hipStream_t st)
{
    hipLaunchKernelGGL((k_compact_edges<1024, 8>), dim3(b.num_scenarios), dim3(1024), 0, st, b.rg_off, rg,
                       ws_edges(ws, L));
}

void launch_edge_boxes(const wm_batch &b, unsigned char *ws, const WsLayout &L, hipStream_t st)
{
    hipLaunchKernelGGL(k_edge_boxes, dim3(b.num_scenarios), dim3(256), 0, st, b.rg_off, ws_edges(ws, L));
}

void launch_build_units(const wm_batch &b, int U, const int32_t *ecount, unsigned char *ws, const WsLayout &L,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_build_units, dim3(1), dim3(1024), 0, st, b.obj_off, ecount, b.num_scenarios, U,
                       (int32_t *)(ws + L.uoff), (int2 *)(ws + L.units), (int32_t *)(ws + L.counter));
}

void launch_dynamics(const wm_batch &b, const StepArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_dynamics, dim3(b.num_scenarios), dim3(128), 0, st, a);
}

void launch_reward(const wm_batch &b, const uint8_t *col, const uint8_t *off, float *reward, hipStream_t st)
{
    hipLaunchKernelGGL(k_reward, dim3(b.num_scenarios), dim3(256), 0, st, b.obj_off, col, off, reward);
}

void launch_inverse(int n, const wm_state &cur, const wm_state &nxt, float dt, float *accel, float *curv,
                    uint8_t *vout, hipStream_t st)
{
    hipLaunchKernelGGL(k_inverse, dim3((n + 255) / 256), dim3(256), 0, st, n, cur, nxt, dt, accel, curv, vout);
}

void launch_overlap(const wm_batch &b, const OverlapArgs &a, hipStream_t st)
{
    const size_t lds = objects_lds(a.maxN) + 256 * sizeof(float);
    const int slices = (b.max_objects + a.U - 1) / a.U;
    if (lds > 65536)
        // a failure here makes the launch below fail, which the caller reports
        (void)hipFuncSetAttribute((const void *)k_overlap, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_overlap, dim3(b.num_scenarios, slices), dim3(256), lds, st, a);
}

static size_t offroad_scratch(int G, int CW) { return scan_lds_bytes(G, CW) + (size_t)256 * CW * 8; }

void launch_offroad(const wm_batch &b, const OffroadArgs &a, hipStream_t st)
{
    const int slices = (b.max_objects + 64 * a.CW - 1) / (64 * a.CW);
    if (64 * a.CW * a.G <= 512) {
        // the pruned scan: objects, scan region, results, boxes, bounds,
        // keys, order and the group counter
        const size_t lds = objects_lds(64 * a.CW) + scan_pruned_lds_bytes(a.G, a.CW, 0) + (size_t)256 * a.CW * 8 +
                           (size_t)kLdsBoxChunks * 80 + (size_t)64 * a.CW * 40 + 16;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)k_offroad_pruned, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds);
        hipLaunchKernelGGL(k_offroad_pruned, dim3(b.num_scenarios, slices), dim3(64 * a.CW * a.G), lds, st, a);
        return;
    }
    const size_t lds = objects_lds(64 * a.CW) + offroad_scratch(a.G, a.CW);
    if (lds > 65536)
        // a failure here makes the launch below fail, which the caller reports
        (void)hipFuncSetAttribute((const void *)k_offroad, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_offroad, dim3(b.num_scenarios, slices), dim3(64 * a.CW * a.G), lds, st, a);
}

size_t rollout_lds_bytes(int maxN, int G, int CW)
{
    const int nthr = 64 * CW * G;
    const size_t idm = (size_t)maxN * 12 + align_up((size_t)maxN, 16) + (size_t)maxN * 12 +
                       (maxN <= kIdmMaskMaxN ? (size_t)maxN * ((maxN + 31) / 32) * 4 : 0);
    // boxes, previous nearest points, keys, order, group counter; the packed
    // boxes of the overlap
    const size_t prune = (size_t)kLdsBoxChunks * 80 + (size_t)64 * CW * 40 + 16 + 16 +
                         (maxN <= kPackedMaxN ? (size_t)maxN * 32 + 16 : 0);
    return objects_lds(maxN) + rollout_scan_bytes(G, CW, maxN) + (size_t)256 * CW * 8 + (size_t)nthr * 4 + 16 * 4 +
           align_up(idm, 16) + prune;
}

void launch_idm_paths(int n, int T, const wm_state &log, const uint8_t *controlled, float4 *path, uint8_t *agent,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_idm_paths, dim3((n + 255) / 256), dim3(256), 0, st, n, T, log, controlled, path, agent);
}

int rollout_grid(int G, int CW, int maxN, int n_units_bound)
{
    // resident work-groups per device for this launch shape; queried once per
    // (device, shape) so that later calls (e.g. under graph capture) make no
    // runtime queries
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, long> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const auto key = std::make_tuple(dev, G, CW, maxN);
    long grid = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end())
            grid = it->second;
    }
    if (grid == 0) {
        const int nthr = 64 * CW * G;
        const size_t lds = rollout_lds_bytes(maxN, G, CW);
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)k_rollout, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rollout, nthr, lds) != hipSuccess || per_cu < 1)
            per_cu = 1;
        int cus = 0;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus < 1)
            cus = 1;
        grid = (long)per_cu * cus;
        std::lock_guard<std::mutex> lk(mu);
        cache[key] = grid;
    }
    return (int)(grid < n_units_bound ? grid : (n_units_bound < 1 ? 1 : n_units_bound));
}

void launch_rollout(const RollArgs &a, int grid, hipStream_t st)
{
    const size_t lds = rollout_lds_bytes(a.maxN, a.G, a.CW);
    // set on every launch: the limit is per function, and an earlier launch
    // of another shape may have lowered it (a host-side call, not a stream
    // operation, so graph capture is unaffected)
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_rollout, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_rollout, dim3(grid), dim3(64 * a.CW * a.G), lds, st, a);
}

void launch_loss_reduce(int S, const int32_t *uoff, const float *lossp, float *loss, hipStream_t st)
{
    hipLaunchKernelGGL(k_loss_reduce, dim3((S + 255) / 256), dim3(256), 0, st, S, uoff, lossp, loss);
}

// ---------------------------------------------------------------------------
// Device-resident workspace of wm_step_noalloc, for callers that cannot
// allocate: WM_NOALLOC_SCRATCH_BYTES per device, held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[WM_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(unsigned char **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static unsigned char *ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        ptr[dev] = (unsigned char *)p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

} // namespace wm
