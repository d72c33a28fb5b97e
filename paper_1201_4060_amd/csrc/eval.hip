// Evaluation on the GPU: position -> cell/offset, Morton binning, and the
// per-particle gather + tensor contraction (Sections 2, 3, 5; Table 1).
#include <algorithm>

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

__global__ void k_debug_cells(CellArgs a, int32_t* cell, double* t) {
    const long p = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (p >= a.P) return;
    const int n[3] = {a.n0, a.n1, a.n2};
    const double ih[3] = {a.ih0, a.ih1, a.ih2};
    int c[3];
    double tt[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) ok = cell_of(a.pos[3 * p + d], ih[d], n[d], c[d], tt[d]) && ok;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        cell[3 * p + d] = ok ? c[d] : -1;
        t[3 * p + d] = ok ? tt[d] : __builtin_nan("");
    }
}

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

__global__ void k_bin_count(CellArgs a, int tile, uint32_t nbuckets_finite, uint32_t* __restrict__ hist,
                            uint32_t* __restrict__ key, uint32_t* __restrict__ rank) {
    const long p = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (p >= a.P) return;
    const int n[3] = {a.n0, a.n1, a.n2};
    const double ih[3] = {a.ih0, a.ih1, a.ih2};
    int c[3];
    double tt[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) ok = cell_of(a.pos[3 * p + d], ih[d], n[d], c[d], tt[d]) && ok;
    uint32_t k = nbuckets_finite;  // overflow bucket for non-finite particles
    if (ok)
        k = (spread3(uint32_t(c[0] / tile)) << 2) | (spread3(uint32_t(c[1] / tile)) << 1) |
            spread3(uint32_t(c[2] / tile));
    key[p] = k;
    rank[p] = atomicAdd(&hist[k], 1u);
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

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_sums(const uint32_t* __restrict__ in, long n,
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
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_top(uint32_t* sums, int m) {
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

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const uint32_t* __restrict__ in, long n,
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

__global__ void k_bin_scatter(long P, const uint32_t* __restrict__ key, const uint32_t* __restrict__ rank,
                              const uint32_t* __restrict__ offs, uint32_t* __restrict__ perm) {
    const long p = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (p >= P) return;
    perm[offs[key[p]] + rank[p]] = uint32_t(p);
}

__global__ void k_fill_u32(uint32_t* p, long n, uint32_t v) {
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x)
        p[i] = v;
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

// w_j(t) = sum_i M[j][i] t^i and w'_j(t) = sum_i M1[j][i] t^i (Horner), M from
// the Section 7 general formula at compile time.
template <int N, typename AT>
__device__ __forceinline__ void bspline_weights(AT t, AT* w, AT* wd) {
    constexpr BSpline<N> B{};
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

struct GatherArgs {
    const void* grid;
    const double* pos;
    const uint32_t* perm;    // binned order, or nullptr
    const uint32_t* hist;    // particles per bucket (tiled kernel)
    const uint32_t* offs;    // first binned index per bucket (tiled kernel)
    void* u;
    void* grad;
    unsigned long long* nonfinite;
    long P;
    int n0, n1, n2;
    int P1, P2;  // padded extents of axes 1 and 2
    double ih0, ih1, ih2;
    int xcd_remap;
    uint32_t nbuckets_finite;
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
__device__ __forceinline__ bool particle_setup(const GatherArgs& a, long p, int* cell, AT (*w)[N],
                                               AT (*wd)[N]) {
    const int n[3] = {a.n0, a.n1, a.n2};
    const double ih[3] = {a.ih0, a.ih1, a.ih2};
    double t[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) ok = cell_of(a.pos[3 * p + d], ih[d], n[d], cell[d], t[d]) && ok;
    if (!ok) return false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        bspline_weights<N, AT>(AT(t[d]), w[d], wd[d]);
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

template <int N, typename CT, typename AT, int C, bool GRAD, int IA0, int IA1, bool FENCE = false,
          typename RowFn>
__device__ __forceinline__ void contract_part(const AT (*w)[N], const AT (*wd)[N], RowFn row,
                                              Partial<AT, C>& out) {
#pragma unroll
    for (int c = 0; c < C; ++c) out.u[c] = out.g0[c] = out.g1[c] = out.g2[c] = AT(0);
#pragma unroll
    for (int ia = IA0; ia < IA1; ++ia) {
        AT v[C], v1[C], v2[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = v1[c] = v2[c] = AT(0);
#pragma unroll
        for (int ib = 0; ib < N; ++ib) {
            const auto* r = row(ia, ib);
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
            // LDS rows: keep one row's values live at a time (bounded registers)
            if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            out.u[c] += w[0][ia] * v[c];
            if constexpr (GRAD) {
                out.g0[c] += wd[0][ia] * v[c];
                out.g1[c] += w[0][ia] * v1[c];
                out.g2[c] += w[0][ia] * v2[c];
            }
        }
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
    contract_part<N, CT, AT, C, GRAD, 0, N / 2, FENCE>(w, wd, row, lo);
    contract_part<N, CT, AT, C, GRAD, N / 2, N, FENCE>(w, wd, row, hi);
    store_sum<AT, C, GRAD>(a, p, lo, hi);
}

// Direct variant: one thread per particle, stencil rows read from global
// memory (caches provide the reuse between neighbouring binned particles).
template <int N, typename CT, int C, bool GRAD>
__global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
    using AT = typename Acc<CT>::type;
    const long j = logical_block(a.xcd_remap) * blockDim.x + threadIdx.x;
    if (j >= a.P) return;
    const long p = a.perm ? long(a.perm[j]) : j;
    int cell[3];
    AT w[3][N], wd[3][N];
    if (!particle_setup<N, AT>(a, p, cell, w, wd)) {
        write_nan<AT, C, GRAD>(a, p);
        atomicAdd(a.nonfinite, 1ull);
        return;
    }
    const CT* base = static_cast<const CT*>(a.grid) +
                     ((long(cell[0]) * a.P1 + cell[1]) * a.P2 + cell[2]) * C;
    const long rowA = long(a.P1) * a.P2 * C;
    const long rowB = long(a.P2) * C;
    contract_and_store<N, CT, AT, C, GRAD>(a, p, w, wd,
                                           [&](int ia, int ib) { return base + ia * rowA + ib * rowB; });
}

__device__ __forceinline__ uint32_t compact3(uint32_t v) {  // inverse of spread3
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x000003ffu;
    return v;
}

template <int N, typename CT, int C, int T>
struct TileGeom {
    static constexpr int R = T + N - 1;               // LDS block edge (points)
    static constexpr int ROW = R * C;                 // elements per LDS row
    static constexpr int ELEMS = R * R * ROW;
    static constexpr int BYTES = ELEMS * int(sizeof(CT));
};

template <typename AT>
__device__ __forceinline__ AT shfl_xor1(AT v) {
    return __shfl_xor(v, 1, 64);
}

// LDS-tiled variant: one 64-lane workgroup per Morton tile of T^3 cells.  The
// tile's (T+N-1)^3 block of the ghost-padded grid is staged in LDS with
// coalesced loads (compile-time geometry, loads issued back to back), then the
// tile's binned particles are evaluated from LDS: one lane per particle, or
// two lanes per particle (one half of the axis-0 sum each, combined with a
// lane shuffle) when the tile holds at most 32 particles.
template <int N, typename CT, int C, bool GRAD, int T>
__global__ __launch_bounds__(64) void k_gather_tiled(GatherArgs a) {
    using AT = typename Acc<CT>::type;
    using G = TileGeom<N, CT, C, T>;
    // Loads: lane = (sub-row, element); one pass covers RPP rows of ROW
    // elements; all rows of one r0-plane are issued before their LDS stores.
    static_assert(G::ROW <= 64, "tile row wider than a wavefront");
    constexpr int RPP = 64 / G::ROW;
    constexpr int NR = (G::R + RPP - 1) / RPP;
    __shared__ CT tile[G::ELEMS];
    const int lane = threadIdx.x;
    const uint32_t bucket = uint32_t(logical_block(a.xcd_remap));
    const uint32_t count = a.hist[bucket];
    if (count == 0) return;
    const uint32_t start = a.offs[bucket];
    if (bucket == a.nbuckets_finite) {  // particles without a cell
        for (uint32_t j = lane; j < count; j += 64) write_nan<AT, C, GRAD>(a, long(a.perm[start + j]));
        if (lane == 0) atomicAdd(a.nonfinite, (unsigned long long)count);
        return;
    }
    const int o0 = int(compact3(bucket >> 2)) * T;
    const int o1 = int(compact3(bucket >> 1)) * T;
    const int o2 = int(compact3(bucket)) * T;
    // valid extent of the block (the last tile along an axis may be partial)
    const int lim0 = a.n0 + N - 1 - o0;        // rows r0 < lim0 exist in the padded grid
    const int lim1 = a.n1 + N - 1 - o1;
    const int limE = (a.n2 + N - 1 - o2) * C;  // elements e < limE exist in a row
    const CT* g = static_cast<const CT*>(a.grid) + (long(o0) * a.P1 + o1) * long(a.P2) * C + long(o2) * C;
    // offsets inside one tile block stay below 2^31 (R * P1 * P2 * C elements)
    const int pitch1 = a.P2 * C;
    const int pitch0 = a.P1 * pitch1;
    // Every lane loads unconditionally; positions outside the padded grid (only
    // in partial tiles, and never read by a particle) load the tile origin.
    const int sub = lane / G::ROW;
    const int e = lane - sub * G::ROW;
    if (sub < RPP) {
        const bool e_ok = e < limE;
        const int lane_off = sub * pitch1 + e;
        const int step = RPP * pitch1;
        const int r0n = min(G::R, lim0);
        for (int r0 = 0; r0 < r0n; ++r0) {
            const int base0 = r0 * pitch0 + lane_off;
            CT v[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                const int r1 = k * RPP + sub;
                const bool ok = e_ok && r1 < lim1 && r1 < G::R;
                v[k] = g[ok ? base0 + k * step : 0];
            }
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                const int r1 = k * RPP + sub;
                if (r1 < G::R) tile[(r0 * G::R + r1) * G::ROW + e] = v[k];
            }
        }
    }
    __syncthreads();
    auto particle_rows = [&](const int* cell) {
        const CT* base = tile + ((cell[0] - o0) * G::R + (cell[1] - o1)) * G::ROW + (cell[2] - o2) * C;
        return [base](int ia, int ib) { return base + (ia * G::R + ib) * G::ROW; };
    };
    if (count <= 32) {
        const uint32_t j = uint32_t(lane >> 1);
        const int half = lane & 1;
        const bool active = j < count;
        const long p = active ? long(a.perm[start + j]) : 0;
        int cell[3] = {o0, o1, o2};
        AT w[3][N], wd[3][N];
        if (active) particle_setup<N, AT>(a, p, cell, w, wd);
        else {
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int k = 0; k < N; ++k) w[d][k] = wd[d][k] = AT(0);
        }
        const auto rows = particle_rows(cell);
        Partial<AT, C> mine, other;
        if (half == 0) contract_part<N, CT, AT, C, GRAD, 0, N / 2, true>(w, wd, rows, mine);
        else contract_part<N, CT, AT, C, GRAD, N / 2, N, true>(w, wd, rows, mine);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            other.u[c] = shfl_xor1(mine.u[c]);
            other.g0[c] = shfl_xor1(mine.g0[c]);
            other.g1[c] = shfl_xor1(mine.g1[c]);
            other.g2[c] = shfl_xor1(mine.g2[c]);
        }
        if (active && half == 0) store_sum<AT, C, GRAD>(a, p, mine, other);
    } else {
        for (uint32_t j = lane; j < count; j += 64) {
            const long p = long(a.perm[start + j]);
            int cell[3];
            AT w[3][N], wd[3][N];
            particle_setup<N, AT>(a, p, cell, w, wd);  // finite by construction of the bucket
            contract_and_store<N, CT, AT, C, GRAD, true>(a, p, w, wd, particle_rows(cell));
        }
    }
}

// ------------------------------------------------------------- launchers ---

namespace {

CellArgs cell_args(const bsi_field* f, const double* pos, long P) {
    CellArgs a;
    a.pos = pos;
    a.P = P;
    a.n0 = f->n[0];
    a.n1 = f->n[1];
    a.n2 = f->n[2];
    a.ih0 = f->inv_h[0];
    a.ih1 = f->inv_h[1];
    a.ih2 = f->inv_h[2];
    return a;
}

template <int N, typename CT, int C>
void launch_gather_t(const GatherArgs& ga, bool grad, unsigned nb, unsigned block, hipStream_t s) {
    if (grad)
        hipLaunchKernelGGL((k_gather<N, CT, C, true>), dim3(nb), dim3(block), 0, s, ga);
    else
        hipLaunchKernelGGL((k_gather<N, CT, C, false>), dim3(nb), dim3(block), 0, s, ga);
}

template <typename CT>
void launch_gather_ct(int N, int C, const GatherArgs& ga, bool grad, unsigned nb, unsigned block,
                      hipStream_t s) {
    if (N == 4) {
        if (C == 1) launch_gather_t<4, CT, 1>(ga, grad, nb, block, s);
        else launch_gather_t<4, CT, 3>(ga, grad, nb, block, s);
    } else {
        if (C == 1) launch_gather_t<6, CT, 1>(ga, grad, nb, block, s);
        else launch_gather_t<6, CT, 3>(ga, grad, nb, block, s);
    }
}

constexpr int TILE_LDS_LIMIT = 64 * 1024;

template <int N, typename CT, int C, int T>
bool launch_tiled_T(const GatherArgs& ga, bool grad, unsigned nb, unsigned block, hipStream_t s) {
    if constexpr (TileGeom<N, CT, C, T>::BYTES > TILE_LDS_LIMIT) {
        return false;
    } else {
        (void)block;
        if (grad)
            hipLaunchKernelGGL((k_gather_tiled<N, CT, C, true, T>), dim3(nb), dim3(64), 0, s, ga);
        else
            hipLaunchKernelGGL((k_gather_tiled<N, CT, C, false, T>), dim3(nb), dim3(64), 0, s, ga);
        return true;
    }
}

template <int N, typename CT, int C>
bool launch_tiled_c(int T, const GatherArgs& ga, bool grad, unsigned nb, unsigned block, hipStream_t s) {
    switch (T) {
        case 4: return launch_tiled_T<N, CT, C, 4>(ga, grad, nb, block, s);
        case 6: return launch_tiled_T<N, CT, C, 6>(ga, grad, nb, block, s);
        case 8: return launch_tiled_T<N, CT, C, 8>(ga, grad, nb, block, s);
        case 10: return launch_tiled_T<N, CT, C, 10>(ga, grad, nb, block, s);
        case 12: return launch_tiled_T<N, CT, C, 12>(ga, grad, nb, block, s);
        case 16: return launch_tiled_T<N, CT, C, 16>(ga, grad, nb, block, s);
        default: return false;
    }
}

template <typename CT>
bool launch_tiled_ct(int N, int C, int T, const GatherArgs& ga, bool grad, unsigned nb, unsigned block,
                     hipStream_t s) {
    if (N == 4)
        return C == 1 ? launch_tiled_c<4, CT, 1>(T, ga, grad, nb, block, s)
                      : launch_tiled_c<4, CT, 3>(T, ga, grad, nb, block, s);
    return C == 1 ? launch_tiled_c<6, CT, 1>(T, ga, grad, nb, block, s)
                  : launch_tiled_c<6, CT, 3>(T, ga, grad, nb, block, s);
}

}  // namespace

size_t bin_bucket_count(const bsi_field* f, int tile) {
    int bits = 0;
    for (int d = 0; d < 3; ++d) {
        const int nt = (f->n[d] + tile - 1) / tile;
        int b = 0;
        while ((1 << b) < nt) ++b;
        bits = std::max(bits, b);
    }
    return size_t(1) << (3 * bits);
}

// Bucket arrays live at the start of the binning scratch: hist[nb], offs[nb], ...
bsi_status bin_run(bsi_field* f, const double* pos, long P, int tile, uint32_t* perm, void* scratch,
                   hipStream_t s) {
    const size_t nbf = bin_bucket_count(f, tile);
    const size_t nb = nbf + 1;
    uint32_t* hist = static_cast<uint32_t*>(scratch);
    uint32_t* offs = hist + nb;
    const size_t nsums = (nb + SCAN_CHUNK - 1) / SCAN_CHUNK;
    uint32_t* sums = offs + nb;
    uint32_t* key = sums + nsums;
    uint32_t* rank = key + P;
    const unsigned fillb = unsigned(std::min<size_t>((nb + 255) / 256, 4096));
    hipLaunchKernelGGL(k_fill_u32, dim3(fillb), dim3(256), 0, s, hist, long(nb), 0u);
    const CellArgs ca = cell_args(f, pos, P);
    const unsigned pb = unsigned((P + 255) / 256);
    {
        StageTimer tm(f->ctx, "bin_count", s);
        hipLaunchKernelGGL(k_bin_count, dim3(pb), dim3(256), 0, s, ca, tile, uint32_t(nbf), hist, key, rank);
    }
    {
        StageTimer tm(f->ctx, "bin_scan", s);
        hipLaunchKernelGGL(k_scan_sums, dim3(unsigned(nsums)), dim3(SCAN_BLOCK), 0, s, hist, long(nb), sums);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_BLOCK), 0, s, sums, int(nsums));
        hipLaunchKernelGGL(k_scan_apply, dim3(unsigned(nsums)), dim3(SCAN_BLOCK), 0, s, hist, long(nb), sums,
                           offs);
    }
    {
        StageTimer tm(f->ctx, "bin_scatter", s);
        hipLaunchKernelGGL(k_bin_scatter, dim3(pb), dim3(256), 0, s, P, key, rank, offs, perm);
    }
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

size_t bin_scratch_bytes(const bsi_field* f, long P, int tile) {
    const size_t nb = bin_bucket_count(f, tile) + 1;
    const size_t nsums = (nb + SCAN_CHUNK - 1) / SCAN_CHUNK;
    return (2 * nb + nsums + 2 * size_t(P)) * sizeof(uint32_t);
}

bool tiled_supported(const bsi_field* f, int tile) {
    const size_t bytes = size_t(tile + f->N - 1) * (tile + f->N - 1) * (tile + f->N - 1) * f->C *
                         dtype_size(f->desc.coef);
    const bool listed = tile == 4 || tile == 6 || tile == 8 || tile == 10 || tile == 12 || tile == 16;
    return listed && bytes <= size_t(TILE_LDS_LIMIT);
}

bsi_status eval_run(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                    const bsi_eval_config& cfg, hipStream_t s) {
    if (P == 0) return BSI_OK;
    int block = cfg.block > 0 ? cfg.block : 256;
    BSI_CHECK(block % 64 == 0 && block >= 64 && block <= 256, BSI_E_INVAL,
              "eval block must be 64, 128, 192 or 256");
    const uint32_t* perm = nullptr;
    const uint32_t* hist = nullptr;
    const uint32_t* offs = nullptr;
    int tile = cfg.sort_tile;
    size_t nbf = 0;
    if (tile > 0) {
        // keep the bucket table at most 2^24 entries
        const int nmax = std::max(f->n[0], std::max(f->n[1], f->n[2]));
        tile = std::max(tile, (nmax + 255) / 256);
        const size_t need = size_t(P) * sizeof(uint32_t) + bin_scratch_bytes(f, P, tile);
        void* ws = nullptr;
        BSI_TRY(get_workspace(f->ctx->eval_ws, s, need, &ws));
        uint32_t* pm = static_cast<uint32_t*>(ws);
        BSI_TRY(bin_run(f, pos, P, tile, pm, pm + P, s));
        perm = pm;
        hist = pm + P;
        nbf = bin_bucket_count(f, tile);
        offs = hist + nbf + 1;
    }
    GatherArgs ga;
    ga.grid = f->grid;
    ga.pos = pos;
    ga.perm = perm;
    ga.hist = hist;
    ga.offs = offs;
    ga.u = u;
    ga.grad = grad;
    ga.nonfinite = f->counters;
    ga.P = P;
    ga.n0 = f->n[0];
    ga.n1 = f->n[1];
    ga.n2 = f->n[2];
    ga.P1 = f->P[1];
    ga.P2 = f->P[2];
    ga.ih0 = f->inv_h[0];
    ga.ih1 = f->inv_h[1];
    ga.ih2 = f->inv_h[2];
    ga.xcd_remap = (perm && cfg.xcd_remap) ? 1 : 0;
    ga.nbuckets_finite = uint32_t(nbf);
    const bool g = grad != nullptr;
    StageTimer tm(f->ctx, "gather", s);
    const bool tiled = perm && cfg.variant == 0 && tiled_supported(f, tile);
    if (tiled) {
        const unsigned nb = unsigned(nbf + 1);
        bool ok = false;
        if (f->desc.coef == BSI_F64) ok = launch_tiled_ct<double>(f->N, f->C, tile, ga, g, nb, block, s);
        else if (f->desc.coef == BSI_F32) ok = launch_tiled_ct<float>(f->N, f->C, tile, ga, g, nb, block, s);
        else ok = launch_tiled_ct<uint16_t>(f->N, f->C, tile, ga, g, nb, block, s);
        BSI_CHECK(ok, BSI_E_UNSUPPORTED, "no tiled gather instance for this tile size");
    } else {
        const unsigned nb = unsigned((P + block - 1) / block);
        if (f->desc.coef == BSI_F64) launch_gather_ct<double>(f->N, f->C, ga, g, nb, block, s);
        else if (f->desc.coef == BSI_F32) launch_gather_ct<float>(f->N, f->C, ga, g, nb, block, s);
        else launch_gather_ct<uint16_t>(f->N, f->C, ga, g, nb, block, s);
    }
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

bsi_status debug_cells_run(bsi_field* f, const double* pos, int64_t P, int32_t* cell, double* t,
                           hipStream_t s) {
    if (P == 0) return BSI_OK;
    const CellArgs ca = cell_args(f, pos, P);
    hipLaunchKernelGGL(k_debug_cells, dim3(unsigned((P + 255) / 256)), dim3(256), 0, s, ca, cell, t);
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

}  // namespace bsi
