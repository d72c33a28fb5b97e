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
    const uint32_t* perm;  // binned order, or nullptr
    void* u;
    void* grad;
    unsigned long long* nonfinite;
    long P;
    int n0, n1, n2;
    int P1, P2;  // padded extents of axes 1 and 2
    double ih0, ih1, ih2;
    int xcd_remap;
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

// One thread per particle.  Contraction order (Table 1 idea: reduce the tensor
// order as early as possible): each contiguous row of N points along axis 2 is
// reduced with w2 and w2' first, then axis 1 with w1 / w1', then axis 0.
template <int N, typename CT, int C, bool GRAD>
__global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
    using AT = typename Acc<CT>::type;
    const long j = logical_block(a.xcd_remap) * blockDim.x + threadIdx.x;
    if (j >= a.P) return;
    const long p = a.perm ? long(a.perm[j]) : j;
    const int n[3] = {a.n0, a.n1, a.n2};
    const double ih[3] = {a.ih0, a.ih1, a.ih2};
    int cell[3];
    double t[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) ok = cell_of(a.pos[3 * p + d], ih[d], n[d], cell[d], t[d]) && ok;
    AT* u = static_cast<AT*>(a.u) + p * C;
    AT* g = GRAD ? static_cast<AT*>(a.grad) + p * C * 3 : nullptr;
    if (!ok) {
        const AT nan = AT(__builtin_nan(""));
#pragma unroll
        for (int c = 0; c < C; ++c) u[c] = nan;
        if constexpr (GRAD) {
#pragma unroll
            for (int c = 0; c < 3 * C; ++c) g[c] = nan;
        }
        atomicAdd(a.nonfinite, 1ull);
        return;
    }
    AT w[3][N], wd[3][N];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        bspline_weights<N, AT>(AT(t[d]), w[d], wd[d]);
        const AT s = AT(ih[d]);
#pragma unroll
        for (int k = 0; k < N; ++k) wd[d][k] *= s;
    }
    const CT* base = static_cast<const CT*>(a.grid) +
                     ((long(cell[0]) * a.P1 + cell[1]) * a.P2 + cell[2]) * C;
    const long rowA = long(a.P1) * a.P2 * C;
    const long rowB = long(a.P2) * C;
    AT acc_u[C], acc_g0[C], acc_g1[C], acc_g2[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc_u[c] = acc_g0[c] = acc_g1[c] = acc_g2[c] = AT(0);
#pragma unroll
    for (int ia = 0; ia < N; ++ia) {
        AT v[C], v1[C], v2[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = v1[c] = v2[c] = AT(0);
#pragma unroll
        for (int ib = 0; ib < N; ++ib) {
            const CT* row = base + ia * rowA + ib * rowB;
            CT raw[N * C];
#pragma unroll
            for (int e = 0; e < N * C; ++e) raw[e] = row[e];
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
            acc_u[c] += w[0][ia] * v[c];
            if constexpr (GRAD) {
                acc_g0[c] += wd[0][ia] * v[c];
                acc_g1[c] += w[0][ia] * v1[c];
                acc_g2[c] += w[0][ia] * v2[c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) u[c] = acc_u[c];
    if constexpr (GRAD) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            g[3 * c + 0] = acc_g0[c];
            g[3 * c + 1] = acc_g1[c];
            g[3 * c + 2] = acc_g2[c];
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
    hipLaunchKernelGGL(k_bin_count, dim3(pb), dim3(256), 0, s, ca, tile, uint32_t(nbf), hist, key, rank);
    hipLaunchKernelGGL(k_scan_sums, dim3(unsigned(nsums)), dim3(SCAN_BLOCK), 0, s, hist, long(nb), sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_BLOCK), 0, s, sums, int(nsums));
    hipLaunchKernelGGL(k_scan_apply, dim3(unsigned(nsums)), dim3(SCAN_BLOCK), 0, s, hist, long(nb), sums,
                       offs);
    hipLaunchKernelGGL(k_bin_scatter, dim3(pb), dim3(256), 0, s, P, key, rank, offs, perm);
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

size_t bin_scratch_bytes(const bsi_field* f, long P, int tile) {
    const size_t nb = bin_bucket_count(f, tile) + 1;
    const size_t nsums = (nb + SCAN_CHUNK - 1) / SCAN_CHUNK;
    return (2 * nb + nsums + 2 * size_t(P)) * sizeof(uint32_t);
}

bsi_status eval_run(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                    const bsi_eval_config& cfg, hipStream_t s) {
    if (P == 0) return BSI_OK;
    int block = cfg.block > 0 ? cfg.block : 256;
    BSI_CHECK(block % 64 == 0 && block >= 64 && block <= 256, BSI_E_INVAL,
              "eval block must be 64, 128, 192 or 256");
    const uint32_t* perm = nullptr;
    int tile = cfg.sort_tile;
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
    }
    GatherArgs ga;
    ga.grid = f->grid;
    ga.pos = pos;
    ga.perm = perm;
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
    const unsigned nb = unsigned((P + block - 1) / block);
    const bool g = grad != nullptr;
    if (f->desc.coef == BSI_F64) launch_gather_ct<double>(f->N, f->C, ga, g, nb, block, s);
    else if (f->desc.coef == BSI_F32) launch_gather_ct<float>(f->N, f->C, ga, g, nb, block, s);
    else launch_gather_ct<uint16_t>(f->N, f->C, ga, g, nb, block, s);
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
