// Device-side building blocks of the evaluation shared by the single-field
// kernels (eval.hip) and the persistent multi-field kernel (batch.hip):
// position -> cell/offset, Morton keys, prefix scans, B-spline weights and the
// per-particle tensor contraction (Sections 2, 3, 5; Table 1).  Both callers
// run exactly these functions, so a particle's result does not depend on which
// kernel evaluated it.
#pragma once

#include <utility>

#include "common.hpp"

namespace bsi {

// ---------------------------------------------------------- cell / offset ---
// Section 5 stencil rule in grid units: s = x * (n/L) as one FP64 product,
// f = floor(s), t = s - f, cell = f mod n (exact Euclidean remainder).
// Contraction is off so that s - f is not fused into an FMA with x * inv_h.
// Returns false when s is not finite.
__device__ __forceinline__ bool cell_of(double x, double inv_h, int n, int& cell, double& t) {
#pragma clang fp contract(off)
    const double s = x * inv_h;
    if (!isfinite(s)) return false;
    const double f = floor(s);
    t = s - f;
    if (f >= 0.0 && f < double(n)) {     // the usual case: x already in [0, L)
        cell = int(f);
        return true;
    }
    if (fabs(f) < 9007199254740992.0) {  // |f| < 2^53: exact in int64
        long long m = static_cast<long long>(f) % n;
        if (m < 0) m += n;
        cell = int(m);
    } else {                             // f = integer-valued double, fmod is exact
        double r = fmod(f, double(n));
        if (r < 0) r += double(n);
        cell = int(r);
    }
    return true;
}

struct CellArgs {
    const double* pos;
    long P;
    int n0, n1, n2;
    double ih0, ih1, ih2;
};

// ---------------------------------------------------------------- binning ---
// Particles are counting-sorted by the Morton code of the tile (cell / T) that
// holds their cell; non-finite particles go to one extra bucket at the end.

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t compact3(uint32_t v) {  // inverse of spread3
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x000003ffu;
    return v;
}

// Exclusive scan of hist[0..n) in three steps: per-block sums, a single-block
// scan of those sums, per-block scan plus offset.
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_CHUNK = SCAN_BLOCK * SCAN_ITEMS;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
    // Hillis-Steele in LDS over SCAN_BLOCK threads
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        const uint32_t add = tid >= off ? sh[tid - off] : 0u;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    const uint32_t incl = sh[tid];
    *total = sh[SCAN_BLOCK - 1];
    __syncthreads();
    return incl - v;
}

static __global__ __launch_bounds__(SCAN_BLOCK) void k_scan_sums(const uint32_t* __restrict__ in, long n,
                                                          uint32_t* __restrict__ sums) {
    __shared__ uint32_t sh[SCAN_BLOCK];
    const long base = long(blockIdx.x) * SCAN_CHUNK + threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += in[base + i];
    uint32_t total;
    block_exclusive_scan(s, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// single block: exclusive scan of sums[0..m) in place (m <= SCAN_BLOCK * items)
static __global__ __launch_bounds__(SCAN_BLOCK) void k_scan_top(uint32_t* sums, int m) {
    __shared__ uint32_t sh[SCAN_BLOCK];
    const int per = (m + SCAN_BLOCK - 1) / SCAN_BLOCK;
    const int beg = threadIdx.x * per;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i)
        if (beg + i < m) s += sums[beg + i];
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sh, &total);
    for (int i = 0; i < per; ++i)
        if (beg + i < m) {
            const uint32_t v = sums[beg + i];
            sums[beg + i] = run;
            run += v;
        }
}

static __global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const uint32_t* __restrict__ in, long n,
                                                           const uint32_t* __restrict__ sums,
                                                           uint32_t* __restrict__ out) {
    __shared__ uint32_t sh[SCAN_BLOCK];
    const long base = long(blockIdx.x) * SCAN_CHUNK + threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sh, &total) + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

static __global__ void k_fill_u32(uint32_t* p, long n, uint32_t v) {
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x)
        p[i] = v;
}

// 16 bytes as a native vector (loads and stores of it are single instructions,
// never aggregate copies) and a load of it from global memory.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u32x4 global_u32x4;

__device__ __forceinline__ u32x4 load_global16(const u32x4* p) {
    return *(global_u32x4*)p;
}

// ------------------------------------------------------- grouping by key ---
// Particles are grouped by bucket key with a two-level counting sort that uses
// no per-particle global atomics (their throughput, not the data volume, bounds
// a one-pass counting sort with one atomic per particle).  The keys [0, nbuckets) are
// split into `ncoarse` contiguous coarse ranges of at most GRP_FINE_MAX keys,
// sized by the caller so that each holds a few hundred particles:
//   k_grp_hist    each block of `ipt * GRP_BLOCK` grouping slots computes the
//                 keys, stores them, and counts its slots per coarse range in
//                 LDS; the counts are stored range-major
//   (scan)        exclusive scan of the counts: where each block's particles
//                 of each coarse range go
//   k_grp_coarse  each block scatters its particles into the coarse ranges as
//                 32-byte records (key, index, position), and clears the
//                 per-key counters of the next steps
//   k_grp_plan    one workgroup: each coarse range is cut into chunks of
//                 GRP_CHUNK particles (a crowded range gets many), listed
//                 range by range
//   k_grp_chunk_count  one workgroup per chunk: LDS histogram of its keys,
//                 added to the per-key counters (one atomic per key present)
//   k_grp_table   one workgroup per coarse range: the bucket table (count and
//                 first binned slot of every key of the range, empty keys
//                 included, so the table needs no clearing), and the counters
//                 turned into per-key cursors
//   k_grp_chunk_scatter  one workgroup per chunk: reserves each key's slots
//                 with one atomic on its cursor, then writes the permutation
//                 and the binned positions.
// The order inside a bucket is whatever the atomics give; no result depends
// on it.  Blocks of the two coarse passes are mapped so that each XCD takes
// one contiguous range of slots, which keeps the partial-line writes of one
// coarse range in one L2.
//
// KeySrc::key(i, &k, &c) gives the key and coarse range of grouping slot i,
// or false for a slot that holds no particle (padding); KeySrc::coarse(i, k)
// gives the coarse range of slot i's key k again; KeySrc::fetch(i, &local, x)
// gives the particle of slot i: its index in its own position array and its
// position.  Coarse::range(c, &lo, &hi) gives the keys [lo, hi) of range c.

constexpr int GRP_BLOCK = SCAN_BLOCK;
constexpr uint32_t GRP_FINE_MAX = 8192;      // keys per coarse range: 32 KB of LDS
constexpr uint32_t GRP_COARSE_MAX = 8192;    // coarse ranges: 32 KB of LDS
constexpr uint32_t GRP_NONE = 0xffffffffu;
constexpr uint32_t GRP_CHUNK = 2048;         // particles per chunk of the fine passes
constexpr int GRP_UNROLL = 8;                // slots per thread whose loads overlap in the coarse pass

// A particle on its way to its bucket: key, index in its own position array
// and position, 32 bytes (written and read as two 16-byte vectors).
struct alignas(16) GrpRec {
    uint32_t key, local;
    double x[3];
};
static_assert(sizeof(GrpRec) == 32, "grouping record is two 16-byte vectors");

__device__ __forceinline__ uint32_t grp_block(long nblk) {
    const long b = blockIdx.x;
    const long q = nblk / 8, r = nblk % 8;
    const long x = b % 8, i = b / 8;
    return uint32_t(x * q + (x < r ? x : r) + i);
}

template <typename KeySrc>
static __global__ __launch_bounds__(GRP_BLOCK) void k_grp_hist(KeySrc ks, long nidx, int ipt, uint32_t ncoarse,
                                                              long nblk, uint32_t* __restrict__ key,
                                                              uint32_t* __restrict__ counts) {
    extern __shared__ uint32_t lh[];
    for (uint32_t c = threadIdx.x; c < ncoarse; c += GRP_BLOCK) lh[c] = 0;
    __syncthreads();
    const uint32_t blk = grp_block(nblk);
    const long b0 = long(blk) * ipt * GRP_BLOCK;
    for (int q = 0; q < ipt; ++q) {
        const long i = b0 + long(q) * GRP_BLOCK + threadIdx.x;
        if (i < nidx) {
            uint32_t k, c;
            if (ks.key(i, k, c)) {
                key[i] = k;
                atomicAdd(&lh[c], 1u);
            } else {
                key[i] = GRP_NONE;
            }
        }
    }
    __syncthreads();
    for (uint32_t c = threadIdx.x; c < ncoarse; c += GRP_BLOCK) counts[long(c) * nblk + blk] = lh[c];
}

template <typename KeySrc>
static __global__ __launch_bounds__(GRP_BLOCK) void k_grp_coarse(KeySrc ks, const uint32_t* __restrict__ key,
                                                                long nidx, int ipt, uint32_t ncoarse, long nblk,
                                                                const uint32_t* __restrict__ gscan,
                                                                GrpRec* __restrict__ rec,
                                                                uint32_t* __restrict__ kcount, long nbuckets) {
    extern __shared__ uint32_t cur[];
    for (long k = blockIdx.x * long(GRP_BLOCK) + threadIdx.x; k < nbuckets; k += long(gridDim.x) * GRP_BLOCK)
        kcount[k] = 0;
    const uint32_t blk = grp_block(nblk);
    for (uint32_t c = threadIdx.x; c < ncoarse; c += GRP_BLOCK) cur[c] = gscan[long(c) * nblk + blk];
    __syncthreads();
    const long b0 = long(blk) * ipt * GRP_BLOCK;
    // GRP_UNROLL slots per step: all their loads are issued before any of
    // their records is written
    for (int q0 = 0; q0 < ipt; q0 += GRP_UNROLL) {
        uint32_t k[GRP_UNROLL], local[GRP_UNROLL];
        double x[GRP_UNROLL][3];
#pragma unroll
        for (int u = 0; u < GRP_UNROLL; ++u) {
            const long i = b0 + long(q0 + u) * GRP_BLOCK + threadIdx.x;
            k[u] = q0 + u < ipt && i < nidx ? key[i] : GRP_NONE;
        }
#pragma unroll
        for (int u = 0; u < GRP_UNROLL; ++u)
            if (k[u] != GRP_NONE) ks.fetch(b0 + long(q0 + u) * GRP_BLOCK + threadIdx.x, local[u], x[u]);
#pragma unroll
        for (int u = 0; u < GRP_UNROLL; ++u) {
            if (k[u] == GRP_NONE) continue;
            const long i = b0 + long(q0 + u) * GRP_BLOCK + threadIdx.x;
            const uint32_t d = atomicAdd(&cur[ks.coarse(i, k[u])], 1u);
            u32x4* r = reinterpret_cast<u32x4*>(rec + d);
            const unsigned long long b0x = __double_as_longlong(x[u][0]);
            const unsigned long long b1x = __double_as_longlong(x[u][1]);
            const unsigned long long b2x = __double_as_longlong(x[u][2]);
            r[0] = u32x4{k[u], local[u], uint32_t(b0x), uint32_t(b0x >> 32)};
            r[1] = u32x4{uint32_t(b1x), uint32_t(b1x >> 32), uint32_t(b2x), uint32_t(b2x >> 32)};
        }
    }
}

// Particles [start, end) of coarse range c in the coarse-sorted arrays.
__device__ __forceinline__ void grp_range_span(const uint32_t* gscan, long nblk, uint32_t ncoarse, uint32_t nvalid,
                                               uint32_t c, uint32_t& start, uint32_t& end) {
    start = gscan[long(c) * nblk];
    end = c + 1 < ncoarse ? gscan[long(c + 1) * nblk] : nvalid;
}

// One workgroup of GRP_PLAN_BLOCK threads: chunk lists.  cbase[c] = first
// chunk of range c; chunk g belongs to range crange[g]; *nchunks = number of
// chunks.  Thread t owns the ranges t*GRP_PLAN_PER .. (its range starts are
// loaded together, then scanned over the workgroup).
constexpr int GRP_PLAN_BLOCK = 1024;
constexpr int GRP_PLAN_PER = int(GRP_COARSE_MAX) / GRP_PLAN_BLOCK;

static __global__ __launch_bounds__(GRP_PLAN_BLOCK) void k_grp_plan(const uint32_t* __restrict__ gscan, long nblk,
                                                                   uint32_t ncoarse, uint32_t nvalid,
                                                                   uint32_t* __restrict__ cbase,
                                                                   uint32_t* __restrict__ crange,
                                                                   uint32_t* __restrict__ nchunks) {
    __shared__ uint32_t wsum[GRP_PLAN_BLOCK / 64];
    const uint32_t c0 = threadIdx.x * GRP_PLAN_PER;
    uint32_t st[GRP_PLAN_PER + 1];
#pragma unroll
    for (int q = 0; q <= GRP_PLAN_PER; ++q) {
        const uint32_t c = c0 + q;
        st[q] = c < ncoarse ? gscan[long(c) * nblk] : nvalid;
    }
    uint32_t m[GRP_PLAN_PER];
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < GRP_PLAN_PER; ++q) {
        m[q] = (st[q + 1] - st[q] + GRP_CHUNK - 1) / GRP_CHUNK;
        sum += m[q];
    }
    // exclusive scan of the per-thread sums: within the wavefront by shuffles,
    // then over the wavefront totals
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
#pragma unroll
    for (int w = 0; w < GRP_PLAN_BLOCK / 64; ++w) {
        const uint32_t v = wsum[w];
        wbase += w < wid ? v : 0u;
        total += v;
    }
    uint32_t run = wbase + incl - sum;
#pragma unroll
    for (int q = 0; q < GRP_PLAN_PER; ++q) {
        const uint32_t c = c0 + q;
        if (c < ncoarse) {
            cbase[c] = run;
            for (uint32_t k = 0; k < m[q]; ++k) crange[run + k] = c;
            run += m[q];
        }
    }
    if (threadIdx.x == 0) *nchunks = total;
}

// Chunk g's range, key span and particles [j0, j1); false past the last chunk.
template <typename Coarse>
__device__ __forceinline__ bool grp_chunk(const Coarse& cm, const uint32_t* crange, const uint32_t* cbase,
                                          const uint32_t* nchunks, const uint32_t* gscan, long nblk,
                                          uint32_t ncoarse, uint32_t nvalid, uint32_t g, uint32_t& klo,
                                          uint32_t& khi, uint32_t& j0, uint32_t& j1) {
    if (g >= __builtin_amdgcn_readfirstlane(*nchunks)) return false;
    const uint32_t c = __builtin_amdgcn_readfirstlane(crange[g]);
    const uint32_t q = g - __builtin_amdgcn_readfirstlane(cbase[c]);
    uint32_t st, en;
    grp_range_span(gscan, nblk, ncoarse, nvalid, c, st, en);
    cm.range(c, klo, khi);
    klo = __builtin_amdgcn_readfirstlane(klo);
    khi = __builtin_amdgcn_readfirstlane(khi);
    j0 = __builtin_amdgcn_readfirstlane(st) + q * GRP_CHUNK;
    j1 = min(j0 + GRP_CHUNK, __builtin_amdgcn_readfirstlane(en));
    return true;
}

// LDS histogram lh[0 .. khi - klo) of the keys of particles [j0, j1).
__device__ __forceinline__ void grp_chunk_hist(const GrpRec* __restrict__ rec, uint32_t klo, uint32_t khi,
                                               uint32_t j0, uint32_t j1, uint32_t* lh) {
    const uint32_t nf = khi - klo;
    for (uint32_t f = threadIdx.x; f < nf; f += GRP_BLOCK) lh[f] = 0;
    __syncthreads();
    for (uint32_t j = j0 + threadIdx.x; j < j1; j += GRP_BLOCK) atomicAdd(&lh[rec[j].key - klo], 1u);
    __syncthreads();
}

template <typename Coarse>
static __global__ __launch_bounds__(GRP_BLOCK) void k_grp_chunk_count(
    Coarse cm, const GrpRec* __restrict__ rec, const uint32_t* __restrict__ crange,
    const uint32_t* __restrict__ cbase, const uint32_t* __restrict__ nchunks, const uint32_t* __restrict__ gscan,
    long nblk, uint32_t ncoarse, uint32_t nvalid, uint32_t* __restrict__ kcount) {
    extern __shared__ uint32_t lh[];
    uint32_t klo, khi, j0, j1;
    if (!grp_chunk(cm, crange, cbase, nchunks, gscan, nblk, ncoarse, nvalid, blockIdx.x, klo, khi, j0, j1)) return;
    grp_chunk_hist(rec, klo, khi, j0, j1, lh);
    for (uint32_t f = threadIdx.x; f < khi - klo; f += GRP_BLOCK)
        if (lh[f]) atomicAdd(&kcount[klo + f], lh[f]);
}

// One workgroup per coarse range: bucket table of its keys from the counts,
// which become the keys' cursors (first binned slot).
template <typename Coarse>
static __global__ __launch_bounds__(GRP_BLOCK) void k_grp_table(Coarse cm, const uint32_t* __restrict__ gscan,
                                                               long nblk, uint32_t ncoarse, uint32_t nvalid,
                                                               uint32_t* __restrict__ kcount,
                                                               uint32_t* __restrict__ hist,
                                                               uint32_t* __restrict__ offs) {
    __shared__ uint32_t sh[GRP_BLOCK];
    const uint32_t c = blockIdx.x;
    uint32_t st, en, klo, khi;
    grp_range_span(gscan, nblk, ncoarse, nvalid, c, st, en);
    cm.range(c, klo, khi);
    const uint32_t nf = khi - klo;
    // exclusive scan over the range's keys: thread t owns [t*per, (t+1)*per)
    const uint32_t per = (nf + GRP_BLOCK - 1) / GRP_BLOCK;
    const uint32_t f0 = threadIdx.x * per;
    uint32_t sum = 0;
    for (uint32_t q = 0; q < per; ++q)
        if (f0 + q < nf) sum += kcount[klo + f0 + q];
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, sh, &total) + st;
    for (uint32_t q = 0; q < per; ++q) {
        const uint32_t f = f0 + q;
        if (f < nf) {
            const uint32_t cnt = kcount[klo + f];
            hist[klo + f] = cnt;
            offs[klo + f] = run;
            kcount[klo + f] = run;
            run += cnt;
        }
    }
}

template <typename Coarse>
static __global__ __launch_bounds__(GRP_BLOCK) void k_grp_chunk_scatter(
    Coarse cm, const GrpRec* __restrict__ rec, const uint32_t* __restrict__ crange,
    const uint32_t* __restrict__ cbase, const uint32_t* __restrict__ nchunks, const uint32_t* __restrict__ gscan,
    long nblk, uint32_t ncoarse, uint32_t nvalid, uint32_t* __restrict__ kcursor, uint32_t* __restrict__ perm,
    double* __restrict__ pos_sorted) {
    extern __shared__ uint32_t lh[];
    uint32_t klo, khi, j0, j1;
    if (!grp_chunk(cm, crange, cbase, nchunks, gscan, nblk, ncoarse, nvalid, blockIdx.x, klo, khi, j0, j1)) return;
    grp_chunk_hist(rec, klo, khi, j0, j1, lh);
    for (uint32_t f = threadIdx.x; f < khi - klo; f += GRP_BLOCK)
        if (lh[f]) lh[f] = atomicAdd(&kcursor[klo + f], lh[f]);
    __syncthreads();
    for (uint32_t j = j0 + threadIdx.x; j < j1; j += GRP_BLOCK) {
        const u32x4* r = reinterpret_cast<const u32x4*>(rec + j);
        const u32x4 a = load_global16(r), b = load_global16(r + 1);
        const uint32_t d = atomicAdd(&lh[a.x - klo], 1u);
        perm[d] = a.y;
        pos_sorted[3 * long(d)] = __longlong_as_double((long long)(uint64_t(a.z) | (uint64_t(a.w) << 32)));
        pos_sorted[3 * long(d) + 1] = __longlong_as_double((long long)(uint64_t(b.x) | (uint64_t(b.y) << 32)));
        pos_sorted[3 * long(d) + 2] = __longlong_as_double((long long)(uint64_t(b.z) | (uint64_t(b.w) << 32)));
    }
}

// Coarse ranges of a single key space: range c = [c << s, min((c + 1) << s, nb)).
struct ShiftCoarse {
    int s;
    uint32_t nb;
    __device__ __forceinline__ void range(uint32_t c, uint32_t& lo, uint32_t& hi) const {
        lo = c << s;
        hi = min((c + 1) << s, nb);
    }
};

// Shift of ShiftCoarse for P particles over nb keys: about `target`
// particles per coarse range when they are spread evenly, within the LDS
// bounds of both levels.
constexpr uint32_t GRP_TARGET = 512;

inline int grp_shift(uint64_t nb, long P, uint64_t target = GRP_TARGET) {
    int s = 0;
    // smallest s with at most max(P / target, 1) ranges, then the bounds
    const uint64_t want = uint64_t(P) / target > 0 ? uint64_t(P) / target : 1;
    while (((nb + (uint64_t(1) << s) - 1) >> s) > want) ++s;
    while (((nb + (uint64_t(1) << s) - 1) >> s) > GRP_COARSE_MAX) ++s;
    // nb <= GRP_COARSE_MAX * GRP_FINE_MAX keeps both bounds
    while ((uint32_t(1) << s) > GRP_FINE_MAX) --s;
    return s;
}

// Host-side plan of a grouping of `nidx` slots (nvalid of them particles)
// over the keys [0, nbuckets) in `ncoarse` coarse ranges.
struct GrpPlan {
    long nidx = 0;
    uint32_t nvalid = 0;
    uint32_t nbuckets = 0;
    uint32_t ncoarse = 0;   // coarse ranges
    uint32_t fine_max = 0;  // most keys in one coarse range
    int ipt = 1;            // slots per thread of the coarse passes
    long nblk = 0;          // blocks of the coarse passes
    size_t ncounts = 0;     // ncoarse * nblk
    size_t nsums = 0;       // scan partial sums
    uint32_t mmax = 0;      // most chunks of the fine passes
};

inline GrpPlan grp_plan(long nidx, uint32_t nvalid, uint32_t nbuckets, uint32_t ncoarse, uint32_t fine_max) {
    GrpPlan g;
    g.nidx = nidx;
    g.nvalid = nvalid;
    g.nbuckets = nbuckets;
    g.ncoarse = ncoarse > 0 ? ncoarse : 1;
    g.fine_max = fine_max;
    // at least ~512 blocks in the coarse passes, at most 32 slots per thread
    long ipt = (nidx + long(GRP_BLOCK) * 512 - 1) / (long(GRP_BLOCK) * 512);
    g.ipt = int(ipt < 1 ? 1 : (ipt > 32 ? 32 : ipt));
    const long chunk = long(g.ipt) * GRP_BLOCK;
    g.nblk = (nidx + chunk - 1) / chunk;
    if (g.nblk == 0) g.nblk = 1;
    g.ncounts = size_t(g.ncoarse) * size_t(g.nblk);
    g.nsums = (g.ncounts + SCAN_CHUNK - 1) / SCAN_CHUNK;
    // sum over ranges of ceil(n_c / GRP_CHUNK) <= nvalid / GRP_CHUNK + ncoarse
    g.mmax = (nvalid + GRP_CHUNK - 1) / GRP_CHUNK + g.ncoarse;
    return g;
}

// Scratch of a grouping, in uint32 words: records (8 words per particle, at
// the start so that they stay 16-byte aligned), key (nidx), counts and their
// scan (ncounts each), scan sums (nsums), per-key counters (nbuckets), chunk
// lists (ncoarse + mmax) and the chunk count.  The scratch must be 16-byte
// aligned.
inline size_t grp_scratch_words(const GrpPlan& g) {
    return 8 * size_t(g.nvalid) + size_t(g.nidx) + 2 * g.ncounts + g.nsums + g.nbuckets + g.ncoarse + g.mmax + 1;
}

// Device buffers of a grouping, carved from its scratch.
struct GrpBuffers {
    GrpRec* rec;
    uint32_t *key, *counts, *gscan, *sums, *kcount, *cbase, *crange, *nchunks;
};

inline GrpBuffers grp_buffers(const GrpPlan& g, uint32_t* scratch) {
    GrpBuffers b;
    b.rec = reinterpret_cast<GrpRec*>(scratch);
    b.key = scratch + 8 * size_t(g.nvalid);
    b.counts = b.key + g.nidx;
    b.gscan = b.counts + g.ncounts;
    b.sums = b.gscan + g.ncounts;
    b.kcount = b.sums + g.nsums;
    b.cbase = b.kcount + g.nbuckets;
    b.crange = b.cbase + g.ncoarse;
    b.nchunks = b.crange + g.mmax;
    return b;
}

// The three steps of a grouping, enqueued on one stream.  The last writes
// hist/offs (one entry per key), perm and pos_sorted (nvalid slots each).
template <typename KeySrc>
inline void grp_count(const KeySrc& ks, const GrpPlan& g, const GrpBuffers& b, hipStream_t st) {
    hipLaunchKernelGGL((k_grp_hist<KeySrc>), dim3(unsigned(g.nblk)), dim3(GRP_BLOCK),
                       size_t(g.ncoarse) * sizeof(uint32_t), st, ks, g.nidx, g.ipt, g.ncoarse, g.nblk, b.key,
                       b.counts);
}

inline void grp_scan(const GrpPlan& g, const GrpBuffers& b, hipStream_t st) {
    const unsigned ns = unsigned(g.nsums);
    hipLaunchKernelGGL(k_scan_sums, dim3(ns), dim3(SCAN_BLOCK), 0, st, b.counts, long(g.ncounts), b.sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_BLOCK), 0, st, b.sums, int(g.nsums));
    hipLaunchKernelGGL(k_scan_apply, dim3(ns), dim3(SCAN_BLOCK), 0, st, b.counts, long(g.ncounts), b.sums, b.gscan);
}

template <typename KeySrc, typename Coarse>
inline void grp_scatter(const KeySrc& ks, const Coarse& cm, const GrpPlan& g, const GrpBuffers& b, uint32_t* hist,
                        uint32_t* offs, uint32_t* perm, double* pos_sorted, hipStream_t st) {
    const size_t lf = size_t(g.fine_max) * sizeof(uint32_t);
    hipLaunchKernelGGL((k_grp_coarse<KeySrc>), dim3(unsigned(g.nblk)), dim3(GRP_BLOCK),
                       size_t(g.ncoarse) * sizeof(uint32_t), st, ks, b.key, g.nidx, g.ipt, g.ncoarse, g.nblk, b.gscan,
                       b.rec, b.kcount, long(g.nbuckets));
    hipLaunchKernelGGL(k_grp_plan, dim3(1), dim3(GRP_PLAN_BLOCK), 0, st, b.gscan, g.nblk, g.ncoarse, g.nvalid,
                       b.cbase, b.crange, b.nchunks);
    hipLaunchKernelGGL((k_grp_chunk_count<Coarse>), dim3(g.mmax), dim3(GRP_BLOCK), lf, st, cm, b.rec, b.crange,
                       b.cbase, b.nchunks, b.gscan, g.nblk, g.ncoarse, g.nvalid, b.kcount);
    hipLaunchKernelGGL((k_grp_table<Coarse>), dim3(g.ncoarse), dim3(GRP_BLOCK), 0, st, cm, b.gscan, g.nblk,
                       g.ncoarse, g.nvalid, b.kcount, hist, offs);
    hipLaunchKernelGGL((k_grp_chunk_scatter<Coarse>), dim3(g.mmax), dim3(GRP_BLOCK), lf, st, cm, b.rec, b.crange,
                       b.cbase, b.nchunks, b.gscan, g.nblk, g.ncoarse, g.nvalid, b.kcount, perm, pos_sorted);
}

// ----------------------------------------------------------------- gather ---

template <typename CT>
struct Acc {
    using type = float;
};
template <>
struct Acc<double> {
    using type = double;
};

template <typename CT, typename AT>
__device__ __forceinline__ AT widen(CT v) {
    if constexpr (sizeof(CT) == 2) return AT(__uint_as_float(uint32_t(v) << 16));
    else return AT(v);
}

// w_j(t) = sum_i M[j][i] t^i and w'_j(t) = sum_i M1[j][i] t^i (Horner), with
// the matrices of a compile-time table (M from the Section 7 general formula
// for the B-spline).
template <int N, typename AT, typename Tab = BSpline<N>>
__device__ __forceinline__ void bspline_weights(AT t, AT* w, AT* wd) {
    constexpr Tab B{};
#pragma unroll
    for (int j = 0; j < N; ++j) {
        AT acc = AT(B.M[j][N - 1]);
#pragma unroll
        for (int i = N - 2; i >= 0; --i) acc = acc * t + AT(B.M[j][i]);
        w[j] = acc;
        AT dacc = AT(B.M1[j][N - 2]);
#pragma unroll
        for (int i = N - 3; i >= 0; --i) dacc = dacc * t + AT(B.M1[j][i]);
        wd[j] = dacc;
    }
}

// The method's weights (Section 2: w = M tbar, w' = M^(1) tbar): the B-spline
// (the paper's method), Lagrange (N = 2: linear) or, for N = 4, cubic Hermite.
// `basis` is the same for every lane of a launch.
template <int N, typename AT>
__device__ __forceinline__ void basis_weights(int basis, AT t, AT* w, AT* wd) {
    if (basis == BSI_BASIS_LAGRANGE) {
        bspline_weights<N, AT, LagrangeM<N>>(t, w, wd);
    } else {
        if constexpr (N == 4) {
            if (basis == BSI_BASIS_HERMITE) {
                bspline_weights<4, AT, HermiteM>(t, w, wd);
                return;
            }
        }
        bspline_weights<N, AT>(t, w, wd);
    }
}

struct GatherArgs {
    const void* grid;
    const double* pos;
    const uint32_t* perm;    // binned order, or nullptr
    const double* pos_sorted;  // positions in binned order (tiled kernel), or nullptr
    const uint32_t* hist;    // particles per bucket (tiled kernel)
    const uint32_t* offs;    // first binned index per bucket (tiled kernel)
    void* u;
    void* grad;
    unsigned long long* nonfinite;
    long P;
    int n0, n1, n2;
    int P1, P2;  // padded extents of axes 1 and 2
    int pitch2;  // elements between consecutive (p0, p1) rows of the grid
    double ih0, ih1, ih2;
    int xcd_remap;
    uint32_t nbuckets_finite;
    uint32_t tiles_per_group;
    int basis;   // bsi_basis of the field
    int cs;      // stored grid entries per cell along an axis: 1, or 2 for Hermite (direct gather only)
    const u32x4* items;  // work items of the tiled kernel: (bucket, first binned slot, count, 0)
    uint32_t* ctl;       // number of items and the ranges' counters (tiled kernel; ITEM_CTL_WORDS)
};

__device__ __forceinline__ long logical_block(int remap) {
    const long b = blockIdx.x;
    if (!remap) return b;
    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD one
    // contiguous range of logical blocks (a compact region of binned particles).
    const long B = gridDim.x;
    const long q = B / 8, r = B % 8;
    const long x = b % 8, i = b / 8;
    return x * q + (x < r ? x : r) + i;
}

template <typename AT, int C, bool GRAD>
__device__ __forceinline__ void write_nan(const GatherArgs& a, long p) {
    const AT nan = AT(__builtin_nan(""));
    AT* u = static_cast<AT*>(a.u) + p * C;
#pragma unroll
    for (int c = 0; c < C; ++c) u[c] = nan;
    if constexpr (GRAD) {
        AT* g = static_cast<AT*>(a.grad) + p * C * 3;
#pragma unroll
        for (int c = 0; c < 3 * C; ++c) g[c] = nan;
    }
}

// Cell and weights of particle p (Section 5 stencil, Section 2 weights).
template <int N, typename AT>
__device__ __forceinline__ bool particle_setup_x(const GatherArgs& a, const double* x, int* cell,
                                                 AT (*w)[N], AT (*wd)[N]) {
    const int n[3] = {a.n0, a.n1, a.n2};
    const double ih[3] = {a.ih0, a.ih1, a.ih2};
    double t[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) ok = cell_of(x[d], ih[d], n[d], cell[d], t[d]) && ok;
    if (!ok) return false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        basis_weights<N, AT>(a.basis, AT(t[d]), w[d], wd[d]);
        const AT s = AT(ih[d]);
#pragma unroll
        for (int k = 0; k < N; ++k) wd[d][k] *= s;
    }
    return true;
}

// Tensor contraction of the N^3 (x C) local coefficients with the weights.
// Order follows the Table 1 idea (reduce the tensor order as early as
// possible): each contiguous row of N points along axis 2 is reduced with w2
// and w2' first, then axis 1 with w1 / w1', then axis 0.  The axis-0 sum is
// split into two fixed halves (ia < N/2 and ia >= N/2) that are added at the
// end, so that one particle can also be shared by two lanes; every gather
// variant uses exactly this arithmetic, so their results are bitwise equal.
// `row(ia, ib)` returns a pointer to the N*C coefficients of row (ia, ib).
template <typename AT, int C>
struct Partial {
    AT u[C], g0[C], g1[C], g2[C];
};

// One axis-0 plane: rows row(ib), ib < N, reduced along axis 2 then axis 1,
// accumulated into out with the plane's axis-0 weights w0k, wd0k (rows read
// straight from global memory).
template <int N, typename CT, typename AT, int C, bool GRAD, typename PlaneRowFn>
__device__ __forceinline__ void contract_plane(AT w0k, AT wd0k, const AT (*w)[N], const AT (*wd)[N],
                                               PlaneRowFn row, Partial<AT, C>& out) {
    AT v[C], v1[C], v2[C];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = v1[c] = v2[c] = AT(0);
#pragma unroll
    for (int ib = 0; ib < N; ++ib) {
        const CT* r = row(ib);
        CT raw[N * C];
#pragma unroll
        for (int e = 0; e < N * C; ++e) raw[e] = r[e];
        AT tr[C], trd[C];
#pragma unroll
        for (int c = 0; c < C; ++c) tr[c] = trd[c] = AT(0);
#pragma unroll
        for (int e = 0; e < N; ++e) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const AT val = widen<CT, AT>(raw[e * C + c]);
                tr[c] += w[2][e] * val;
                if constexpr (GRAD) trd[c] += wd[2][e] * val;
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            v[c] += w[1][ib] * tr[c];
            if constexpr (GRAD) {
                v1[c] += wd[1][ib] * tr[c];
                v2[c] += w[1][ib] * trd[c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        out.u[c] += w0k * v[c];
        if constexpr (GRAD) {
            out.g0[c] += wd0k * v[c];
            out.g1[c] += w0k * v1[c];
            out.g2[c] += w0k * v2[c];
        }
    }
}

// Raw values of one stencil row (N points x C components along axis 2) held
// in registers between their LDS read and their use.  BF16 rows in LDS start
// on 2-byte boundaries, and unaligned wide LDS reads are slow: they are read
// as aligned dwords from the dword boundary at or below the row start and
// realigned by a funnel shift per pair of values when used.  The N*C/2 + 1
// dwords end at most 4 bytes past the row's values, inside the row's padding
// to whole 16-byte chunks for every tile geometry of the tiled gathers.
// PS is the LDS pitch of one grid point in elements: C for densely packed
// rows; 4 for FP32 three-component points held in 16-byte slots, read with one
// 16-byte LDS read each (element e = point e / 3, component e % 3).
template <int N, typename CT, int C, int PS = C>
struct LdsRow {
    static_assert(PS == C, "padded points: FP32, three components");
    CT raw[N * C];
    __device__ __forceinline__ void load(const CT* r) {
#pragma unroll
        for (int e = 0; e < N * C; ++e) raw[e] = r[e];
    }
    __device__ __forceinline__ CT get(int e) const { return raw[e]; }
};

template <int N>
struct LdsRow<N, float, 3, 4> {
    f32x4 pt[N];
    __device__ __forceinline__ void load(const float* r) {
#pragma unroll
        for (int k = 0; k < N; ++k) pt[k] = *reinterpret_cast<const f32x4*>(r + 4 * k);
    }
    __device__ __forceinline__ float get(int e) const { return pt[e / 3][e % 3]; }
};

template <int N, int C>
struct LdsRow<N, uint16_t, C, C> {
    static_assert((N * C) % 2 == 0, "BF16 rows are read as pairs");
    static constexpr int ND = N * C / 2 + 1;
    uint32_t dw[ND];
    uint32_t mis;  // the row's misalignment in bits: 0 or 16
    __device__ __forceinline__ void load(const uint16_t* r) {
        const uint32_t m = uint32_t(reinterpret_cast<uintptr_t>(r)) & 2u;
        const uint32_t* d = reinterpret_cast<const uint32_t*>(r - (m >> 1));
        mis = m * 8u;
#pragma unroll
        for (int k = 0; k < ND; ++k) dw[k] = d[k];
    }
    __device__ __forceinline__ uint16_t get(int e) const {
        const uint32_t v = __builtin_amdgcn_alignbit(dw[e / 2 + 1], dw[e / 2], mis);
        return uint16_t((e & 1) ? (v >> 16) : (v & 0xffffu));
    }
};

// The axis-1/axis-2 sums of one axis-0 plane: v = sum_ib w1[ib] (sum_e w2[e] row[e]),
// with v1 (w1') and v2 (w2') for the gradient.
template <typename AT, int C>
struct PlaneSum {
    AT v[C], v1[C], v2[C];
};

// PlaneSum of NP consecutive planes from LDS rows row(k, ib), the rows
// software-pipelined as in contract_planes (the same arithmetic, row by row).
template <int N, typename CT, typename AT, int C, bool GRAD, int NP, int PS, typename RowFn>
__device__ __forceinline__ void plane_sums(const AT (*w)[N], const AT (*wd)[N], RowFn row, PlaneSum<AT, C>* V) {
    LdsRow<N, CT, C, PS> buf[2];
    buf[0].load(row(0, 0));
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        AT v[C], v1[C], v2[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = v1[c] = v2[c] = AT(0);
#pragma unroll
        for (int ib = 0; ib < N; ++ib) {
            const int r = k * N + ib;
            if (r + 1 < NP * N) buf[(r + 1) & 1].load(row((r + 1) / N, (r + 1) % N));
            const LdsRow<N, CT, C, PS>& cur = buf[r & 1];
            AT tr[C], trd[C];
#pragma unroll
            for (int c = 0; c < C; ++c) tr[c] = trd[c] = AT(0);
#pragma unroll
            for (int e = 0; e < N; ++e) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const AT val = widen<CT, AT>(cur.get(e * C + c));
                    tr[c] += w[2][e] * val;
                    if constexpr (GRAD) trd[c] += wd[2][e] * val;
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                v[c] += w[1][ib] * tr[c];
                if constexpr (GRAD) {
                    v1[c] += wd[1][ib] * tr[c];
                    v2[c] += w[1][ib] * trd[c];
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if constexpr (GRAD) asm volatile("" : "+v"(v[c]), "+v"(v1[c]), "+v"(v2[c]));
                else asm volatile("" : "+v"(v[c]));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            V[k].v[c] = v[c];
            V[k].v1[c] = v1[c];
            V[k].v2[c] = v2[c];
        }
    }
}

// out += plane k's terms (the accumulation step of contract_planes).
template <typename AT, int C, bool GRAD>
__device__ __forceinline__ void chain_add(Partial<AT, C>& out, AT w0k, AT wd0k, const PlaneSum<AT, C>& V) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
        out.u[c] += w0k * V.v[c];
        if constexpr (GRAD) {
            out.g0[c] += wd0k * V.v[c];
            out.g1[c] += w0k * V.v1[c];
            out.g2[c] += w0k * V.v2[c];
        }
    }
}

template <typename AT, int C, bool GRAD>
__device__ __forceinline__ PlaneSum<AT, C> shfl_planesum(const PlaneSum<AT, C>& V, int src) {
    PlaneSum<AT, C> r;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        r.v[c] = __shfl(V.v[c], src, 64);
        if constexpr (GRAD) {
            r.v1[c] = __shfl(V.v1[c], src, 64);
            r.v2[c] = __shfl(V.v2[c], src, 64);
        }
    }
    return r;
}

template <typename AT, int C, bool GRAD>
__device__ __forceinline__ Partial<AT, C> shfl_partial(const Partial<AT, C>& P, int src) {
    Partial<AT, C> r;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        r.u[c] = __shfl(P.u[c], src, 64);
        if constexpr (GRAD) {
            r.g0[c] = __shfl(P.g0[c], src, 64);
            r.g1[c] = __shfl(P.g1[c], src, 64);
            r.g2[c] = __shfl(P.g2[c], src, 64);
        }
    }
    return r;
}

// NIA consecutive axis-0 planes: w0[k], wd0[k] are the axis-0 weights of
// plane k and row(k, ib) its rows; accumulation order is k = 0..NIA-1.
// FENCE (LDS-resident rows): the NIA*N rows are software-pipelined -- the
// LDS reads of row r+1 are issued before the arithmetic of row r, and a
// scheduling fence after each row keeps at most two rows in registers -- so
// that the LDS latency of one row hides behind the FMAs of the previous one.
// Otherwise (rows in global memory) everything is unrolled and left to the
// compiler.  The arithmetic, and its order, is the same in both forms.
template <int N, typename CT, typename AT, int C, bool GRAD, int NIA, bool FENCE = false, int PS = C,
          typename RowFn>
__device__ __forceinline__ void contract_planes(const AT* w0, const AT* wd0, const AT (*w)[N],
                                                const AT (*wd)[N], RowFn row, Partial<AT, C>& out) {
    static_assert(FENCE || PS == C, "rows in global memory are densely packed");
#pragma unroll
    for (int c = 0; c < C; ++c) out.u[c] = out.g0[c] = out.g1[c] = out.g2[c] = AT(0);
    if constexpr (FENCE) {
        LdsRow<N, CT, C, PS> buf[2];
        buf[0].load(row(0, 0));
#pragma unroll
        for (int k = 0; k < NIA; ++k) {
            AT v[C], v1[C], v2[C];
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = v1[c] = v2[c] = AT(0);
#pragma unroll
            for (int ib = 0; ib < N; ++ib) {
                const int r = k * N + ib;
                if (r + 1 < NIA * N) buf[(r + 1) & 1].load(row((r + 1) / N, (r + 1) % N));
                const LdsRow<N, CT, C, PS>& cur = buf[r & 1];
                AT tr[C], trd[C];
#pragma unroll
                for (int c = 0; c < C; ++c) tr[c] = trd[c] = AT(0);
#pragma unroll
                for (int e = 0; e < N; ++e) {
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const AT val = widen<CT, AT>(cur.get(e * C + c));
                        tr[c] += w[2][e] * val;
                        if constexpr (GRAD) trd[c] += wd[2][e] * val;
                    }
                }
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    v[c] += w[1][ib] * tr[c];
                    if constexpr (GRAD) {
                        v1[c] += wd[1][ib] * tr[c];
                        v2[c] += w[1][ib] * trd[c];
                    }
                }
                // the row's arithmetic is pinned above the fence (the
                // accumulators pass through an empty side-effecting asm);
                // otherwise it may sink below later rows' reads
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if constexpr (GRAD) asm volatile("" : "+v"(v[c]), "+v"(v1[c]), "+v"(v2[c]));
                    else asm volatile("" : "+v"(v[c]));
                }
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                out.u[c] += w0[k] * v[c];
                if constexpr (GRAD) {
                    out.g0[c] += wd0[k] * v[c];
                    out.g1[c] += w0[k] * v1[c];
                    out.g2[c] += w0[k] * v2[c];
                }
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < NIA; ++k)
            contract_plane<N, CT, AT, C, GRAD>(w0[k], wd0[k], w, wd, [&](int ib) { return row(k, ib); }, out);
    }
}

template <typename AT, int C, bool GRAD>
__device__ __forceinline__ void store_sum(const GatherArgs& a, long p, const Partial<AT, C>& lo,
                                          const Partial<AT, C>& hi) {
    AT* u = static_cast<AT*>(a.u) + p * C;
#pragma unroll
    for (int c = 0; c < C; ++c) u[c] = lo.u[c] + hi.u[c];
    if constexpr (GRAD) {
        AT* g = static_cast<AT*>(a.grad) + p * C * 3;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            g[3 * c + 0] = lo.g0[c] + hi.g0[c];
            g[3 * c + 1] = lo.g1[c] + hi.g1[c];
            g[3 * c + 2] = lo.g2[c] + hi.g2[c];
        }
    }
}

template <int N, typename CT, typename AT, int C, bool GRAD, bool FENCE = false, typename RowFn>
__device__ __forceinline__ void contract_and_store(const GatherArgs& a, long p, const AT (*w)[N],
                                                   const AT (*wd)[N], RowFn row) {
    Partial<AT, C> lo, hi;
    contract_planes<N, CT, AT, C, GRAD, N / 2, FENCE>(w[0], wd[0], w, wd, row, lo);
    contract_planes<N, CT, AT, C, GRAD, N / 2, FENCE>(
        w[0] + N / 2, wd[0] + N / 2, w, wd, [&](int k, int ib) { return row(N / 2 + k, ib); }, hi);
    store_sum<AT, C, GRAD>(a, p, lo, hi);
}

// FP32 three-component blocks hold one grid point per 16-byte LDS slot (the
// fourth float is spare): a stencil row is then N aligned 16-byte LDS reads
// wherever it starts, where densely packed 12-byte points need 4-byte reads.
template <typename CT, int C>
constexpr bool padded_points() {
    return sizeof(CT) == 4 && C == 3;
}

// Lanes per particle for sparse boxes (0: none): order 6 -> three lanes of
// two axis-0 planes each, order 4 -> four lanes of one plane each.
template <int N>
constexpr int split_lanes() {
    return N == 6 ? 3 : (N == 4 ? 4 : 0);
}

// LDS copy of the (T0+N-1) x (T1+N-1) x (T2+N-1) block of grid points that
// the particles of a T0 x T1 x T2 cell box read: rows along axis 2, either
// packed densely and padded to whole 16-byte chunks (PAD false), or one
// 16-byte slot per point (PAD true).
template <int N, typename CT, int C, int T0, int T1, int T2, bool PAD = padded_points<CT, C>()>
struct BlockGeom {
    static_assert(!PAD || padded_points<CT, C>(), "padded points: FP32, three components");
    static constexpr bool PADDED = PAD;
    static constexpr int R0 = T0 + N - 1;
    static constexpr int R1 = T1 + N - 1;
    static constexpr int R2 = T2 + N - 1;
    static constexpr int VEC = 16 / int(sizeof(CT));                // elements per 16-byte slot
    static constexpr int PS = PAD ? VEC : C;                        // LDS pitch of a point (elements)
    static constexpr int CH = PAD ? R2 : (R2 * C + VEC - 1) / VEC;  // 16-byte slots per row
    static constexpr int LROW = CH * VEC;                           // LDS row pitch (elements)
    static constexpr int ROWS = R0 * R1;
    static constexpr int SLOTS = ROWS * CH;
    static constexpr int BYTES = SLOTS * 16;
    // packed rows are copied in 16-byte chunks from the block origin, which
    // must then start on a 16-byte boundary inside a grid row; padded points
    // are copied one point (4-byte aligned) per slot
    static constexpr bool ALIGNED = PAD || (T2 * C * int(sizeof(CT))) % 16 == 0;
};

// Cubic Morton tiles of T^3 cells.
template <int N, typename CT, int C, int T, bool PAD = padded_points<CT, C>()>
using TileGeom = BlockGeom<N, CT, C, T, T, T, PAD>;


template <typename AT>
__device__ __forceinline__ AT shfl_xor1(AT v) {
    return __shfl_xor(v, 1, 64);
}

// Barrier for LDS only: orders the wavefront's LDS accesses without waiting for
// outstanding global loads (the next tile's prefetch stays in flight).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint32_t next_tile(const GatherArgs& a, uint32_t b, uint32_t end) {
    while (b < end && a.hist[b] == 0) ++b;
    return b;
}

// Requests the LDS copy of the block of geometry G with cell origin (o0, o1,
// o2) in the ghost-padded grid (row pitch pitch2 elements, P1 rows per plane):
// slots tid, tid + B, ... are copied global -> LDS by the DMA path of the load
// unit (no registers hold the data), each wavefront's instruction q filling 64
// consecutive 16-byte slots from its wave-uniform LDS base; only the last step
// can reach past the block, and its lanes there are masked off.  A packed slot
// is the row's next 16-byte chunk; a padded slot is the 16 bytes from its
// point's first element (the point and the first element of the next one).
// Rows outside the padded grid (partial blocks only; never read by a
// particle) load the block origin instead; reads past a row's end land in the
// next row, its pitch padding or the allocation's slack.  Does not wait for
// the loads.
template <int N, typename CT, int C, typename G, int B>
__device__ __forceinline__ void block_dma(const CT* grid, int n0, int n1, int P1, long pitch2, int o0, int o1,
                                          int o2, u32x4* lds) {
    constexpr int PERB = (G::SLOTS + B - 1) / B;
    const int tid = threadIdx.x;
    const int lim0 = n0 + N - 1 - o0;
    const int lim1 = n1 + N - 1 - o1;
    const CT* g = grid + (long(o0) * P1 + o1) * pitch2 + long(o2) * C;
    // offsets inside a block stay < 2^31 elements
    const int p1e = int(pitch2);
    const int p0e = P1 * p1e;
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
#pragma unroll
    for (int q = 0; q < PERB; ++q) {
        const int sl = q * B + tid;
        const int row = sl / G::CH;
        const int ch = sl - row * G::CH;
        const int r0 = row / G::R1;
        const int r1 = row - r0 * G::R1;
        const bool ok = r0 < lim0 && r1 < lim1;
        const int e = ok ? r0 * p0e + r1 * p1e + ch * (G::PADDED ? C : G::VEC) : 0;
        if (q < PERB - 1 || sl < G::SLOTS)
            __builtin_amdgcn_global_load_lds((global_u32x4*)(g + e),
                                             (__attribute__((address_space(3))) void*)(lds + q * B + wbase),
                                             16, 0, 0);
    }
}

// One particle evaluated straight from the grid in global memory (the caches
// provide the reuse between neighbouring binned particles).  j is the
// particle's slot in binned order, or its index when the particles are not
// binned; positions come from the binned copy when there is one.
template <int N, typename CT, int C, bool GRAD>
__device__ __forceinline__ void direct_eval(const GatherArgs& a, long j) {
    using AT = typename Acc<CT>::type;
    const long p = a.perm ? long(a.perm[j]) : j;
    const double* xp = a.pos_sorted ? a.pos_sorted + 3 * j : a.pos + 3 * p;
    const double x[3] = {xp[0], xp[1], xp[2]};
    int cell[3];
    AT w[3][N], wd[3][N];
    if (!particle_setup_x<N, AT>(a, x, cell, w, wd)) {
        write_nan<AT, C, GRAD>(a, p);
        atomicAdd(a.nonfinite, 1ull);
    } else {
        const CT* base = static_cast<const CT*>(a.grid) + (long(a.cs * cell[0]) * a.P1 + a.cs * cell[1]) * a.pitch2 +
                         long(a.cs * cell[2]) * C;
        const long rowA = long(a.P1) * a.pitch2;
        const long rowB = a.pitch2;
        Partial<AT, C> lo, hi;
        auto row = [&](int ia, int ib) { return base + ia * rowA + ib * rowB; };
        contract_planes<N, CT, AT, C, GRAD, N / 2>(w[0], wd[0], w, wd, row, lo);
        contract_planes<N, CT, AT, C, GRAD, N / 2>(w[0] + N / 2, wd[0] + N / 2, w, wd,
                                                   [&](int k, int ib) { return row(N / 2 + k, ib); }, hi);
        store_sum<AT, C, GRAD>(a, p, lo, hi);
    }
}

// The aligned dword reads of a BF16 row (contract_plane) stay inside the row's
// LDS pitch for every stencil start dc = 0 .. T2-1 of a T2-cell box.
template <int N, int C, int T2, int LROW>
constexpr bool bf16_rows_fit() {
    for (int dc = 0; dc < T2; ++dc) {
        const int start = 2 * dc * C;
        if (start - start % 4 + 4 * (N * C / 2 + 1) > 2 * LROW) return false;
    }
    return true;
}

// LDS bytes one workgroup of B threads needs for the block geometry G: the
// block itself (lanes past its last slot load nothing), so that as many blocks
// as possible fit a CU (six of 27 KB for order 6 with 8^3 tiles).
template <typename G, int B>
constexpr int block_lds_bytes() {
    return G::SLOTS * 16;
}

template <int N, typename CT, int C, int T, int B>
constexpr int tile_lds_bytes() {
    return block_lds_bytes<TileGeom<N, CT, C, T>, B>();
}

// The `count` particles from binned slot `start`, all with cells inside the
// box of geometry G at cell origin (o0, o1, o2), evaluated by one workgroup
// of B threads from an LDS copy of the box's block of the grid.  All 16-byte
// loads of the block are issued at once (one memory round trip) straight into
// `lds` (block_lds_bytes() of it); with `fill` false the LDS already holds the
// block (the previous call was for the same box).  Lanes per particle: three
// (order 6; four for order 4) when a round holds all the particles, each lane
// summing its axis-0 planes and the lanes of planes 0 and N/2 gathering the
// rest of their half by lane shuffles; else two (one half of the axis-0 sum
// each) up to B/2 particles; else one.  Every mode adds the same terms in the
// same order.  Every thread of the workgroup calls this with the same
// arguments.
template <int N, typename CT, int C, bool GRAD, typename G, int B>
__device__ __forceinline__ void block_eval_cells(const GatherArgs& a, int o0, int o1, int o2, uint32_t count,
                                                 uint32_t start, u32x4* lds, bool fill = true) {
    using AT = typename Acc<CT>::type;
    static_assert(sizeof(CT) != 2 || bf16_rows_fit<N, C, G::R2 - N + 1, G::LROW>(),
                  "BF16 row reads would leave the LDS row");
    const CT* tile = reinterpret_cast<const CT*>(lds);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // a sparse box is split: SL lanes per particle (split_lanes), else two
    // lanes per particle up to half a workgroup of particles, else one
    constexpr int SL = split_lanes<N>();
    constexpr int SPW = SL > 0 ? 64 / SL : 1;  // particles per wavefront when split
    const bool split = SL > 0 && count <= uint32_t(SPW * (B / 64));
    const bool pair = !split && count <= uint32_t(B / 2);
    const int ppw = split ? SPW : (pair ? 32 : 64);  // particles per wavefront and round
    const int stride = ppw * (B / 64);
    const uint32_t jlane = split ? uint32_t((tid >> 6) * SPW + lane / (SL > 0 ? SL : 1))
                                 : (pair ? uint32_t(tid >> 1) : uint32_t(tid));
    const int part = split ? lane % (SL > 0 ? SL : 1) : (pair ? (tid & 1) : 0);
    const int half = part;
    const bool lane_ok = !split || lane < SPW * SL;  // the spare lane of a split wavefront
    if (count == 0) return;  // uniform: no barrier is skipped by part of the workgroup
    // per-lane particle state of one round: slot, position, stencil origin
    // in the block and the weights
    long p;
    bool active;
    double x[3];
    int cell[3];
    AT w[3][N], wd[3][N];
    auto fetch_round = [&](uint32_t j0) {
        const uint32_t j = j0 + jlane;
        active = j < count && lane_ok;
        const uint32_t jj = start + (active ? j : 0u);
        p = long(a.perm[jj]);
        x[0] = a.pos_sorted[3 * long(jj)];
        x[1] = a.pos_sorted[3 * long(jj) + 1];
        x[2] = a.pos_sorted[3 * long(jj) + 2];
    };
    // finite by construction of the bucket
    auto setup_round = [&]() { particle_setup_x<N, AT>(a, x, cell, w, wd); };
    // the first round's particles are requested before the block, so that one
    // memory round trip serves both (4 % faster for order 6)
    fetch_round(0);
    {
        if (fill)
            block_dma<N, CT, C, G, B>(static_cast<const CT*>(a.grid), a.n0, a.n1, a.P1, long(a.pitch2), o0, o1, o2,
                                      lds);
        // the weights' arithmetic stays below every block load: the compiler
        // waits for all loads in flight before the first use of a position,
        // so arithmetic scheduled between the block loads would split them
        // into two round trips
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);  // every counter at zero: the block is in LDS
    }
    setup_round();
    lds_barrier();
    for (uint32_t j0 = 0;;) {
        // a wavefront without any particle in this round skips it (uniform);
        // inside a working wavefront, lanes past the end evaluate the box's
        // first particle and store nothing
        if (j0 + uint32_t(ppw * (tid / 64)) < count) {
            const CT* base =
                tile + ((cell[0] - o0) * G::R1 + (cell[1] - o1)) * G::LROW + (cell[2] - o2) * G::PS;
            auto rows = [base](int ia, int ib) { return base + (ia * G::R1 + ib) * G::LROW; };
            bool done = false;
            if constexpr (SL > 0) {
                if (split) {
                    // lane `part` takes planes part*PPL .. part*PPL + PPL - 1; the
                    // lanes holding planes 0 and N/2 gather the other planes of
                    // their half and add them up in the order of contract_planes
                    constexpr int PPL = N / SL;
                    PlaneSum<AT, C> V[PPL];
                    plane_sums<N, CT, AT, C, GRAD, PPL, G::PS>(
                        w, wd, [&](int k, int ib) { return rows(part * PPL + k, ib); }, V);
                    Partial<AT, C> lo, hi;
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        lo.u[c] = lo.g0[c] = lo.g1[c] = lo.g2[c] = AT(0);
                        hi.u[c] = hi.g0[c] = hi.g1[c] = hi.g2[c] = AT(0);
                    }
                    if constexpr (N == 6) {
                        // part 0: planes 0, 1 (+ 2 from part 1); part 2: (3 from part 1 +) 4, 5
                        const PlaneSum<AT, C> X = shfl_planesum<AT, C, GRAD>(V[0], (lane + 1) & 63);
                        const PlaneSum<AT, C> Y = shfl_planesum<AT, C, GRAD>(V[1], (lane + 63) & 63);
                        chain_add<AT, C, GRAD>(lo, w[0][0], wd[0][0], V[0]);
                        chain_add<AT, C, GRAD>(lo, w[0][1], wd[0][1], V[1]);
                        chain_add<AT, C, GRAD>(lo, w[0][2], wd[0][2], X);
                        chain_add<AT, C, GRAD>(hi, w[0][3], wd[0][3], Y);
                        chain_add<AT, C, GRAD>(hi, w[0][4], wd[0][4], V[0]);
                        chain_add<AT, C, GRAD>(hi, w[0][5], wd[0][5], V[1]);
                    } else {
                        // part 0: plane 0 (+ 1 from part 1); part 2: plane 2 (+ 3 from part 3)
                        static_assert(N == 4, "split lanes for orders 4 and 6");
                        const PlaneSum<AT, C> X = shfl_planesum<AT, C, GRAD>(V[0], (lane + 1) & 63);
                        chain_add<AT, C, GRAD>(lo, w[0][0], wd[0][0], V[0]);
                        chain_add<AT, C, GRAD>(lo, w[0][1], wd[0][1], X);
                        chain_add<AT, C, GRAD>(hi, w[0][2], wd[0][2], V[0]);
                        chain_add<AT, C, GRAD>(hi, w[0][3], wd[0][3], X);
                    }
                    const Partial<AT, C> H = shfl_partial<AT, C, GRAD>(hi, (lane + 2) & 63);
                    if (active && part == 0) store_sum<AT, C, GRAD>(a, p, lo, H);
                    done = true;
                }
            }
            if (done) {
            } else if (pair) {
                // both lanes of a pair run the same instructions: lane `half`
                // takes planes half*N/2 .. half*N/2 + N/2 - 1
                const int ia0 = half * (N / 2);
                AT w0s[N / 2], wd0s[N / 2];
#pragma unroll
                for (int k = 0; k < N / 2; ++k) {
                    w0s[k] = half ? w[0][N / 2 + k] : w[0][k];
                    wd0s[k] = half ? wd[0][N / 2 + k] : wd[0][k];
                }
                Partial<AT, C> mine, other;
                contract_planes<N, CT, AT, C, GRAD, N / 2, true, G::PS>(
                    w0s, wd0s, w, wd, [&](int k, int ib) { return rows(ia0 + k, ib); }, mine);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    other.u[c] = shfl_xor1(mine.u[c]);
                    other.g0[c] = shfl_xor1(mine.g0[c]);
                    other.g1[c] = shfl_xor1(mine.g1[c]);
                    other.g2[c] = shfl_xor1(mine.g2[c]);
                }
                if (active && half == 0) store_sum<AT, C, GRAD>(a, p, mine, other);
            } else {
                Partial<AT, C> lo, hi;
                contract_planes<N, CT, AT, C, GRAD, N / 2, true, G::PS>(w[0], wd[0], w, wd, rows, lo);
                contract_planes<N, CT, AT, C, GRAD, N / 2, true, G::PS>(
                    w[0] + N / 2, wd[0] + N / 2, w, wd, [&](int k, int ib) { return rows(N / 2 + k, ib); },
                    hi);
                if (active) store_sum<AT, C, GRAD>(a, p, lo, hi);
            }
        }
        j0 += uint32_t(stride);
        if (j0 >= count) break;
        fetch_round(j0);
        setup_round();
    }
    lds_barrier();
}

// NaN outputs for the `count` particles without a cell (the last bucket),
// which are also counted.
template <typename AT, int C, bool GRAD, int B>
__device__ __forceinline__ void nonfinite_eval(const GatherArgs& a, uint32_t count, uint32_t start) {
    for (uint32_t j = threadIdx.x; j < count; j += B) write_nan<AT, C, GRAD>(a, long(a.perm[start + j]));
    if (threadIdx.x == 0) atomicAdd(a.nonfinite, (unsigned long long)count);
}

// The `count` binned particles from slot `start` of bucket `cur` (Morton tile
// `cur` of T^3 cells, or the bucket of particles without a cell when `cur` ==
// nbuckets_finite) evaluated by one workgroup of B threads
// (block_eval_cells); `fill` false: the LDS holds tile `cur`'s block already.
// Every thread of the workgroup must call this with the same arguments.
template <int N, typename CT, int C, bool GRAD, int T, int B>
__device__ __forceinline__ void bucket_eval(const GatherArgs& a, uint32_t cur, uint32_t count, uint32_t start,
                                            u32x4* tile_v, bool fill = true) {
    using AT = typename Acc<CT>::type;
    if (cur == a.nbuckets_finite) {
        nonfinite_eval<AT, C, GRAD, B>(a, count, start);
    } else {
        const int o0 = int(compact3(cur >> 2)) * T;
        const int o1 = int(compact3(cur >> 1)) * T;
        const int o2 = int(compact3(cur)) * T;
        block_eval_cells<N, CT, C, GRAD, TileGeom<N, CT, C, T>, B>(a, o0, o1, o2, count, start, tile_v, fill);
    }
}

// All particles of bucket `cur` (bucket_eval).
template <int N, typename CT, int C, bool GRAD, int T, int B>
__device__ __forceinline__ void tile_eval(const GatherArgs& a, uint32_t cur, u32x4* tile_v) {
    // every value that steers a loop or branch holding a barrier is made
    // wave-uniform explicitly, so that those loops are scalar
    const uint32_t count = __builtin_amdgcn_readfirstlane(a.hist[cur]);
    const uint32_t start = __builtin_amdgcn_readfirstlane(a.offs[cur]);
    bucket_eval<N, CT, C, GRAD, T, B>(a, cur, count, start, tile_v);
}

// ------------------------------------------------------- work items ---------
// The tiled gather's work: every non-empty bucket cut into items of at most
// `chunk` binned particles (in bucket order), so that a crowded tile is shared
// by several workgroups.  The items are split into ITEM_RANGES contiguous ranges (one per
// XCD: neighbouring tiles, whose blocks overlap, meet in the same L2); the
// persistent workgroups of an XCD take the items of its range in order through
// an atomic counter, then those of the other ranges.

constexpr int ITEM_RANGES = 8;
// ctl[0] = item count; the next item of range x at ctl[ITEM_CTL_STRIDE * (x + 1)],
// each counter on a 128-byte line of its own (atomics on one line serialise)
constexpr int ITEM_CTL_STRIDE = 32;
constexpr int ITEM_CTL_WORDS = ITEM_CTL_STRIDE * (ITEM_RANGES + 1);
// items a workgroup takes from a range with one atomic
constexpr uint32_t ITEM_TAKE = 4;

// Items of buckets [b0, b0 + SCAN_ITEMS) of thread t (per-thread counts).
__device__ __forceinline__ uint32_t item_pieces(const uint32_t* __restrict__ hist, long nb, uint32_t chunk, long b0,
                                                uint32_t* cnt, uint32_t* pieces) {
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        cnt[i] = b0 + i < nb ? hist[b0 + i] : 0u;
        pieces[i] = (cnt[i] + chunk - 1) / chunk;
        sum += pieces[i];
    }
    return sum;
}

// Items in bucket order, in three launches: k_item_sums (items per
// SCAN_CHUNK buckets), k_scan_top over those sums, k_items (each workgroup
// scans its buckets' counts from its sum's offset and writes their items; the
// last one also writes the item count ctl[0]).
static __global__ __launch_bounds__(SCAN_BLOCK) void k_item_sums(const uint32_t* __restrict__ hist, long nb,
                                                          uint32_t chunk, uint32_t* __restrict__ sums) {
    __shared__ uint32_t sh[SCAN_BLOCK];
    uint32_t cnt[SCAN_ITEMS], pieces[SCAN_ITEMS];
    const uint32_t s =
        item_pieces(hist, nb, chunk, long(blockIdx.x) * SCAN_CHUNK + threadIdx.x * SCAN_ITEMS, cnt, pieces);
    uint32_t total;
    block_exclusive_scan(s, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

static __global__ __launch_bounds__(SCAN_BLOCK) void k_items(const uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ offs, long nb, uint32_t chunk,
                                                      const uint32_t* __restrict__ sums, u32x4* __restrict__ items,
                                                      uint32_t* ctl) {
    __shared__ uint32_t sh[SCAN_BLOCK];
    const long b0 = long(blockIdx.x) * SCAN_CHUNK + threadIdx.x * SCAN_ITEMS;
    uint32_t cnt[SCAN_ITEMS], pieces[SCAN_ITEMS];
    const uint32_t s = item_pieces(hist, nb, chunk, b0, cnt, pieces);
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sh, &total) + sums[blockIdx.x];
    if (blockIdx.x + 1 == gridDim.x && threadIdx.x == 0) ctl[0] = sums[blockIdx.x] + total;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (pieces[i] == 0) continue;
        const uint32_t st = offs[b0 + i];
        for (uint32_t k = 0; k < pieces[i]; ++k) {
            const uint32_t first = k * chunk;
            items[run + k] = u32x4{uint32_t(b0 + i), st + first, min(chunk, cnt[i] - first), 0u};
        }
        run += pieces[i];
    }
}

// First item of range x of W items.
__device__ __forceinline__ uint32_t item_range_begin(uint32_t W, uint32_t x) {
    return uint32_t((uint64_t(W) * x) / ITEM_RANGES);
}

// Index of the next ITEM_TAKE items of range x, requested by the workgroup's
// first lane (the value is valid in that lane only; item_take_finish makes it
// uniform).
__device__ __forceinline__ uint32_t item_take_issue(uint32_t* ctl, uint32_t x) {
    uint32_t v = 0;
    if (threadIdx.x == 0) v = atomicAdd(ctl + ITEM_CTL_STRIDE * (x + 1), ITEM_TAKE);
    return v;
}

template <int B>
__device__ __forceinline__ uint32_t item_take_finish(uint32_t v, uint32_t* sh) {
    if constexpr (B == 64) {
        return __builtin_amdgcn_readfirstlane(v);
    } else {
        if (threadIdx.x == 0) *sh = v;
        __syncthreads();
        const uint32_t r = __builtin_amdgcn_readfirstlane(*sh);
        __syncthreads();
        return r;
    }
}

}  // namespace bsi
