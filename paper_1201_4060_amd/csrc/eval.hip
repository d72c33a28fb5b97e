// Evaluation on the GPU: position -> cell/offset, Morton binning, and the
// per-particle gather + tensor contraction (Sections 2, 3, 5; Table 1).
#include <algorithm>

#include "gather.hpp"

namespace bsi {

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

// Key of a particle: the Morton index of its sort tile, or nbuckets_finite
// for a non-finite position; its coarse range is key >> shift.
struct MortonKey {
    CellArgs a;
    int tile;
    uint32_t nbuckets_finite;
    int shift;
    __device__ __forceinline__ uint32_t coarse(long, uint32_t k) const { return k >> shift; }
    __device__ __forceinline__ void fetch(long p, uint32_t& local, double* x) const {
        local = uint32_t(p);
        x[0] = a.pos[3 * p];
        x[1] = a.pos[3 * p + 1];
        x[2] = a.pos[3 * p + 2];
    }
    __device__ __forceinline__ bool key(long p, uint32_t& k, uint32_t& cr) const {
        const int n[3] = {a.n0, a.n1, a.n2};
        const double ih[3] = {a.ih0, a.ih1, a.ih2};
        int c[3];
        double tt[3];
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) ok = cell_of(a.pos[3 * p + d], ih[d], n[d], c[d], tt[d]) && ok;
        k = nbuckets_finite;
        if (ok)
            k = (spread3(uint32_t(c[0] / tile)) << 2) | (spread3(uint32_t(c[1] / tile)) << 1) |
                spread3(uint32_t(c[2] / tile));
        cr = k >> shift;
        return true;
    }
};

// ----------------------------------------------------------------- gather ---

// Direct variant: one thread per particle.
template <int N, typename CT, int C, bool GRAD>
__global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
    const long j = logical_block(a.xcd_remap) * blockDim.x + threadIdx.x;
    if (j >= a.P) return;
    direct_eval<N, CT, C, GRAD>(a, j);
}

// LDS-tiled variant: persistent workgroups of B threads evaluate work items
// (pieces of Morton tiles of T^3 cells, k_items).  A workgroup takes the items
// of its home range in order, ITEM_TAKE at a time through the range's
// counter, then those of the other ranges, and ends when every range is
// exhausted; the next take is requested before the last item of the current
// one is evaluated.  Home range: blockIdx % ITEM_RANGES with xcd_remap
// (workgroups are dispatched to the XCDs in turn), 0 for every workgroup
// without.  Consecutive items of one tile reuse the tile's block in LDS.
// (the LDS block limits FP64 and padded FP32 blocks to about one wavefront
// per SIMD: the registers are not the limit there)
template <int N, typename CT, int C, bool GRAD, int T, int B>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(
    sizeof(CT) == 8 || padded_points<CT, C>() ? 1 : 2))) void k_gather_tiled(GatherArgs a) {
    __shared__ u32x4 tile_v[tile_lds_bytes<N, CT, C, T, B>() / 16];
    __shared__ uint32_t taken;
    // every value that steers a loop or branch holding a barrier is made
    // wave-uniform explicitly, so that those loops are scalar
    const uint32_t W = __builtin_amdgcn_readfirstlane(a.ctl[0]);
    const uint32_t home = a.xcd_remap ? uint32_t(blockIdx.x) % ITEM_RANGES : 0u;
    uint32_t prev = 0xffffffffu;  // bucket whose block the LDS holds
    for (uint32_t r = 0; r < ITEM_RANGES; ++r) {
        const uint32_t x = (home + r) % ITEM_RANGES;
        const uint32_t lo = item_range_begin(W, x);
        const uint32_t hi = item_range_begin(W, x + 1);
        uint32_t i = item_take_finish<B>(item_take_issue(a.ctl, x), &taken);
        while (lo + i < hi) {
            const uint32_t m = min(ITEM_TAKE, hi - lo - i);
            uint32_t next = 0;
            for (uint32_t k = 0; k < m; ++k) {
                const u32x4 it = a.items[lo + i + k];
                const uint32_t cur = __builtin_amdgcn_readfirstlane(it.x);
                const uint32_t start = __builtin_amdgcn_readfirstlane(it.y);
                const uint32_t count = __builtin_amdgcn_readfirstlane(it.z);
                if (k + 1 == m) next = item_take_issue(a.ctl, x);
                bucket_eval<N, CT, C, GRAD, T, B>(a, cur, count, start, tile_v, cur != prev);
                prev = cur;
            }
            i = item_take_finish<B>(next, &taken);
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
    if (N == 2) {
        if (C == 1) launch_gather_t<2, CT, 1>(ga, grad, nb, block, s);
        else launch_gather_t<2, CT, 3>(ga, grad, nb, block, s);
    } else if (N == 4) {
        if (C == 1) launch_gather_t<4, CT, 1>(ga, grad, nb, block, s);
        else launch_gather_t<4, CT, 3>(ga, grad, nb, block, s);
    } else {
        if (C == 1) launch_gather_t<6, CT, 1>(ga, grad, nb, block, s);
        else launch_gather_t<6, CT, 3>(ga, grad, nb, block, s);
    }
}

constexpr int TILE_LDS_LIMIT = 64 * 1024;  // static LDS per workgroup

template <int N, typename CT, int C, int T>
constexpr bool tile_ok() {
    return TileGeom<N, CT, C, T>::BYTES <= TILE_LDS_LIMIT && TileGeom<N, CT, C, T>::ALIGNED;
}

// 64 threads for small tiles, 256 for tiles whose block fills the LDS budget
template <int N, typename CT, int C, int T>
constexpr int tile_block() {
    return TileGeom<N, CT, C, T>::SLOTS >= 3072 ? 256 : 64;
}

// The tiled gather runs as many workgroups as can be resident at once (its
// occupancy, asked once per instance, on every CU).
template <int N, typename CT, int C, bool GRAD, int T, int B>
void launch_tiled_kernel(const GatherArgs& ga, int num_cus, hipStream_t s) {
    auto k = k_gather_tiled<N, CT, C, GRAD, T, B>;
    static unsigned nb = 0;
    static std::once_flag once;
    std::call_once(once, [&] {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k, B, 0) != hipSuccess || v < 1) v = 1;
        nb = unsigned(v);
    });
    hipLaunchKernelGGL(k, dim3(nb * unsigned(std::max(num_cus, 1))), dim3(B), 0, s, ga);
}

template <int N, typename CT, int C, int T>
bool launch_tiled_T(const GatherArgs& ga, bool grad, bool wide, int num_cus, hipStream_t s) {
    if constexpr (!tile_ok<N, CT, C, T>()) {
        return false;
    } else {
        constexpr int B = tile_block<N, CT, C, T>();
        if constexpr (T == 8 && B == 64) {
            // dense 8^3 tiles: four wavefronts share one LDS block
            if (wide) {
                if (grad) launch_tiled_kernel<N, CT, C, true, T, 256>(ga, num_cus, s);
                else launch_tiled_kernel<N, CT, C, false, T, 256>(ga, num_cus, s);
                return true;
            }
        }
        if (grad) launch_tiled_kernel<N, CT, C, true, T, B>(ga, num_cus, s);
        else launch_tiled_kernel<N, CT, C, false, T, B>(ga, num_cus, s);
        return true;
    }
}

// threads per workgroup of the tiled gather for this field and tile (0 if no
// tiled instance)
template <int N, typename CT, int C, int T>
constexpr int tiled_block_T(bool wide) {
    if constexpr (!tile_ok<N, CT, C, T>()) return 0;
    else return (T == 8 && tile_block<N, CT, C, T>() == 64 && wide) ? 256 : tile_block<N, CT, C, T>();
}

template <int N, typename CT, int C>
bool launch_tiled_c(int T, const GatherArgs& ga, bool grad, bool wide, int num_cus, hipStream_t s) {
    switch (T) {
        case 4: return launch_tiled_T<N, CT, C, 4>(ga, grad, wide, num_cus, s);
        case 6: return launch_tiled_T<N, CT, C, 6>(ga, grad, wide, num_cus, s);
        case 8: return launch_tiled_T<N, CT, C, 8>(ga, grad, wide, num_cus, s);
        case 12: return launch_tiled_T<N, CT, C, 12>(ga, grad, wide, num_cus, s);
        case 16: return launch_tiled_T<N, CT, C, 16>(ga, grad, wide, num_cus, s);
        default: return false;
    }
}

template <typename CT>
bool launch_tiled_ct(int N, int C, int T, const GatherArgs& ga, bool grad, bool wide, int num_cus,
                     hipStream_t s) {
    if (N == 2) {   // linear: 8^3-cell tiles only
        if (T != 8) return false;
        return C == 1 ? launch_tiled_T<2, CT, 1, 8>(ga, grad, wide, num_cus, s)
                      : launch_tiled_T<2, CT, 3, 8>(ga, grad, wide, num_cus, s);
    }
    if (N == 4)
        return C == 1 ? launch_tiled_c<4, CT, 1>(T, ga, grad, wide, num_cus, s)
                      : launch_tiled_c<4, CT, 3>(T, ga, grad, wide, num_cus, s);
    return C == 1 ? launch_tiled_c<6, CT, 1>(T, ga, grad, wide, num_cus, s)
                  : launch_tiled_c<6, CT, 3>(T, ga, grad, wide, num_cus, s);
}

template <int N, typename CT, int C>
int tiled_block_c(int T, bool wide) {
    switch (T) {
        case 4: return tiled_block_T<N, CT, C, 4>(wide);
        case 6: return tiled_block_T<N, CT, C, 6>(wide);
        case 8: return tiled_block_T<N, CT, C, 8>(wide);
        case 12: return tiled_block_T<N, CT, C, 12>(wide);
        case 16: return tiled_block_T<N, CT, C, 16>(wide);
        default: return 0;
    }
}

template <typename CT>
int tiled_block_ct(int N, int C, int T, bool wide) {
    if (N == 2) {
        if (T != 8) return 0;
        return C == 1 ? tiled_block_T<2, CT, 1, 8>(wide) : tiled_block_T<2, CT, 3, 8>(wide);
    }
    if (N == 4) return C == 1 ? tiled_block_c<4, CT, 1>(T, wide) : tiled_block_c<4, CT, 3>(T, wide);
    return C == 1 ? tiled_block_c<6, CT, 1>(T, wide) : tiled_block_c<6, CT, 3>(T, wide);
}

template <int N, typename CT, int C>
bool tile_ok_rt(int T) {
    switch (T) {
        case 4: return tile_ok<N, CT, C, 4>();
        case 6: return tile_ok<N, CT, C, 6>();
        case 8: return tile_ok<N, CT, C, 8>();
        case 12: return tile_ok<N, CT, C, 12>();
        case 16: return tile_ok<N, CT, C, 16>();
        default: return false;
    }
}

template <typename CT>
bool tile_ok_ct(int N, int C, int T) {
    if (N == 2) return T == 8 && (C == 1 ? tile_ok<2, CT, 1, 8>() : tile_ok<2, CT, 3, 8>());
    if (N == 4) return C == 1 ? tile_ok_rt<4, CT, 1>(T) : tile_ok_rt<4, CT, 3>(T);
    return C == 1 ? tile_ok_rt<6, CT, 1>(T) : tile_ok_rt<6, CT, 3>(T);
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

// At most 2^24 + 1 keys (effective_tile).
static GrpPlan bin_plan(const bsi_field* f, long P, int tile, int* shift) {
    const uint64_t nb = bin_bucket_count(f, tile) + 1;
    *shift = grp_shift(nb, P);
    const uint32_t ncoarse = uint32_t((nb + (uint64_t(1) << *shift) - 1) >> *shift);
    return grp_plan(P, uint32_t(P), uint32_t(nb), ncoarse, uint32_t(std::min<uint64_t>(nb, uint64_t(1) << *shift)));
}

// Workspace of a binned evaluation (16-byte aligned): the grouping scratch,
// then the binned positions (3P doubles), the permutation (P), the bucket
// counts and first slots (nb each).
BinLayout bin_layout(const bsi_field* f, long P, int tile) {
    int shift = 0;
    const size_t nb = bin_bucket_count(f, tile) + 1;
    BinLayout l;
    l.grp = 0;
    l.pos = (grp_scratch_words(bin_plan(f, P, tile, &shift)) * sizeof(uint32_t) + 15) / 16 * 16;
    l.perm = l.pos + 3 * size_t(P) * sizeof(double);
    l.hist = l.perm + size_t(P) * sizeof(uint32_t);
    l.offs = l.hist + nb * sizeof(uint32_t);
    l.bytes = l.offs + nb * sizeof(uint32_t);
    return l;
}

bsi_status bin_run(bsi_field* f, const double* pos, long P, int tile, void* scratch, uint32_t* perm,
                   double* pos_sorted, uint32_t* hist, uint32_t* offs, hipStream_t s) {
    const size_t nbf = bin_bucket_count(f, tile);
    const size_t nb = nbf + 1;
    int shift = 0;
    const GrpPlan g = bin_plan(f, P, tile, &shift);
    const GrpBuffers gb = grp_buffers(g, static_cast<uint32_t*>(scratch));
    const MortonKey mk{cell_args(f, pos, P), tile, uint32_t(nbf), shift};
    {
        StageTimer tm(f->ctx, "bin_count", s);
        grp_count(mk, g, gb, s);
    }
    {
        StageTimer tm(f->ctx, "bin_scan", s);
        grp_scan(g, gb, s);
    }
    {
        StageTimer tm(f->ctx, "bin_scatter", s);
        grp_scatter(mk, ShiftCoarse{shift, uint32_t(nb)}, g, gb, hist, offs, perm, pos_sorted, s);
    }
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

bool tiled_supported(const bsi_field* f, int tile) {
    // Hermite fields (two stored entries per cell and axis) use the direct gather
    if (f->cs != 1) return false;
    if (f->desc.coef == BSI_F64) return tile_ok_ct<double>(f->N, f->C, tile);
    if (f->desc.coef == BSI_F32) return tile_ok_ct<float>(f->N, f->C, tile);
    return tile_ok_ct<uint16_t>(f->N, f->C, tile);
}

// Sort tile actually used: at least n/256 cells per tile edge, so that the
// bucket table has at most 2^24 entries.
static int effective_tile(const bsi_field* f, const bsi_eval_config& cfg) {
    if (cfg.sort_tile <= 0) return 0;
    const int nmax = std::max(f->n[0], std::max(f->n[1], f->n[2]));
    return std::max(cfg.sort_tile, (nmax + 255) / 256);
}

// Threads per workgroup of the tiled gather for field f, tile and config (0:
// no tiled instance, the direct gather runs).
static int tiled_block(const bsi_field* f, int tile, const bsi_eval_config& cfg) {
    if (tile == 0 || cfg.variant != 0 || !tiled_supported(f, tile)) return 0;
    const bool wide = cfg.tile_block == 256;
    if (f->desc.coef == BSI_F64) return tiled_block_ct<double>(f->N, f->C, tile, wide);
    if (f->desc.coef == BSI_F32) return tiled_block_ct<float>(f->N, f->C, tile, wide);
    return tiled_block_ct<uint16_t>(f->N, f->C, tile, wide);
}

// Work items of the tiled gather after the binning's arrays: at most one per
// non-empty bucket plus one per `chunk` particles, 16 bytes each, then the
// control words and the per-group item sums.
struct ItemLayout {
    size_t items, ctl, sums, bytes;
    uint32_t chunk;
};

static ItemLayout item_layout(const bsi_field* f, long P, int tile, const bsi_eval_config& cfg, size_t base) {
    ItemLayout l{};
    const int B = tiled_block(f, tile, cfg);
    l.items = l.ctl = l.bytes = base;
    if (B == 0) return l;
    l.chunk = uint32_t(B) * uint32_t(cfg.item_rounds > 0 ? cfg.item_rounds : 4);
    const size_t nb = bin_bucket_count(f, tile) + 1;
    const size_t cap = nb + size_t(P) / l.chunk + 1;
    l.items = (base + 15) / 16 * 16;
    l.ctl = l.items + cap * 16;
    l.sums = l.ctl + ITEM_CTL_WORDS * sizeof(uint32_t);
    l.bytes = l.sums + (nb + SCAN_CHUNK - 1) / SCAN_CHUNK * sizeof(uint32_t);
    return l;
}

size_t eval_ws_bytes(const bsi_field* f, int64_t P, const bsi_eval_config& cfg) {
    const int tile = effective_tile(f, cfg);
    if (tile == 0 || P == 0) return 0;
    return item_layout(f, P, tile, cfg, bin_layout(f, P, tile).bytes).bytes;
}

bsi_status eval_check_config(const bsi_eval_config& cfg) {
    const int block = cfg.block > 0 ? cfg.block : 256;
    BSI_CHECK(block % 64 == 0 && block >= 64 && block <= 256, BSI_E_INVAL,
              "eval block must be 64, 128, 192 or 256");
    BSI_CHECK(cfg.sort_tile >= 0 && cfg.sort_tile <= 1024, BSI_E_INVAL, "sort_tile out of range");
    BSI_CHECK(cfg.tile_block == 0 || cfg.tile_block == 64 || cfg.tile_block == 256, BSI_E_INVAL,
              "tile_block must be 0, 64 or 256");
    BSI_CHECK(cfg.item_rounds >= 0 && cfg.item_rounds <= 1024, BSI_E_INVAL, "item_rounds must be 0..1024");
    return BSI_OK;
}

// The position-only half of an evaluation: binning and work items into ws
// (nothing without binning).
bsi_status eval_bin_ws(bsi_field* f, const double* pos, int64_t P, const bsi_eval_config& cfg, hipStream_t s,
                       void* ws) {
    const int tile = effective_tile(f, cfg);
    if (P == 0 || tile == 0) return BSI_OK;
    BSI_CHECK(ws != nullptr && reinterpret_cast<uintptr_t>(ws) % 16 == 0, BSI_E_INVAL,
              "binned evaluation needs a 16-byte aligned workspace");
    const BinLayout l = bin_layout(f, P, tile);
    char* w = static_cast<char*>(ws);
    uint32_t* hist = reinterpret_cast<uint32_t*>(w + l.hist);
    uint32_t* offs = reinterpret_cast<uint32_t*>(w + l.offs);
    BSI_TRY(bin_run(f, pos, P, tile, w + l.grp, reinterpret_cast<uint32_t*>(w + l.perm),
                    reinterpret_cast<double*>(w + l.pos), hist, offs, s));
    const ItemLayout il = item_layout(f, P, tile, cfg, l.bytes);
    if (il.chunk > 0) {
        StageTimer tm(f->ctx, "bin_items", s);
        uint32_t* ctl = reinterpret_cast<uint32_t*>(w + il.ctl);
        const long nb = long(bin_bucket_count(f, tile)) + 1;
        const unsigned ng = unsigned((nb + SCAN_CHUNK - 1) / SCAN_CHUNK);
        uint32_t* sums = reinterpret_cast<uint32_t*>(w + il.sums);
        hipLaunchKernelGGL(k_item_sums, dim3(ng), dim3(SCAN_BLOCK), 0, s, hist, nb, il.chunk, sums);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_BLOCK), 0, s, sums, int(ng));
        hipLaunchKernelGGL(k_items, dim3(ng), dim3(SCAN_BLOCK), 0, s, hist, offs, nb, il.chunk, sums,
                           reinterpret_cast<u32x4*>(w + il.items), ctl);
    }
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

// The gather half: reads the binning eval_bin_ws left in ws for the same
// (pos, P, cfg) and the field's current grid.
bsi_status eval_gather_ws(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                          const bsi_eval_config& cfg, hipStream_t s, void* ws) {
    if (P == 0) return BSI_OK;
    const int block = cfg.block > 0 ? cfg.block : 256;
    const int tile = effective_tile(f, cfg);
    GatherArgs ga;
    ga.grid = f->grid;
    ga.pos = pos;
    ga.perm = nullptr;
    ga.pos_sorted = nullptr;
    ga.hist = nullptr;
    ga.offs = nullptr;
    ga.items = nullptr;
    ga.ctl = nullptr;
    size_t nbf = 0;
    ItemLayout il{};
    if (tile > 0) {
        BSI_CHECK(ws != nullptr && reinterpret_cast<uintptr_t>(ws) % 16 == 0, BSI_E_INVAL,
                  "binned evaluation needs a 16-byte aligned workspace");
        const BinLayout l = bin_layout(f, P, tile);
        char* w = static_cast<char*>(ws);
        ga.pos_sorted = reinterpret_cast<const double*>(w + l.pos);
        ga.perm = reinterpret_cast<const uint32_t*>(w + l.perm);
        ga.hist = reinterpret_cast<const uint32_t*>(w + l.hist);
        ga.offs = reinterpret_cast<const uint32_t*>(w + l.offs);
        nbf = bin_bucket_count(f, tile);
        il = item_layout(f, P, tile, cfg, l.bytes);
        if (il.chunk > 0) {
            ga.items = reinterpret_cast<const u32x4*>(w + il.items);
            ga.ctl = reinterpret_cast<uint32_t*>(w + il.ctl);
        }
    }
    ga.u = u;
    ga.grad = grad;
    ga.nonfinite = f->counters;
    ga.P = P;
    ga.n0 = f->n[0];
    ga.n1 = f->n[1];
    ga.n2 = f->n[2];
    ga.P1 = f->P[1];
    ga.P2 = f->P[2];
    ga.pitch2 = f->pitch2;
    ga.tiles_per_group = uint32_t(cfg.tiles_per_group > 0 ? cfg.tiles_per_group : 4);
    ga.ih0 = f->inv_h[0];
    ga.ih1 = f->inv_h[1];
    ga.ih2 = f->inv_h[2];
    ga.xcd_remap = (ga.perm && cfg.xcd_remap) ? 1 : 0;
    ga.nbuckets_finite = uint32_t(nbf);
    ga.basis = f->basis;
    ga.cs = f->cs;
    const bool g = grad != nullptr;
    if (ga.items) {
        // the ranges' counters start at zero for every run over one binning
        StageTimer tm(f->ctx, "bin_items", s);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, ga.ctl + ITEM_CTL_STRIDE,
                           long(ITEM_CTL_WORDS - ITEM_CTL_STRIDE), 0u);
    }
    StageTimer tm(f->ctx, "gather", s);
    if (ga.items) {
        bool ok = false;
        // tile_block 256 asks for four wavefronts per 8^3 tile (dense tiles)
        const bool wide = cfg.tile_block == 256;
        const int ncu = f->ctx->num_cus;
        if (f->desc.coef == BSI_F64) ok = launch_tiled_ct<double>(f->N, f->C, tile, ga, g, wide, ncu, s);
        else if (f->desc.coef == BSI_F32) ok = launch_tiled_ct<float>(f->N, f->C, tile, ga, g, wide, ncu, s);
        else ok = launch_tiled_ct<uint16_t>(f->N, f->C, tile, ga, g, wide, ncu, s);
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

bsi_status eval_run_ws(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                       const bsi_eval_config& cfg, hipStream_t s, void* ws) {
    if (P == 0) return BSI_OK;
    BSI_TRY(eval_check_config(cfg));
    BSI_TRY(eval_bin_ws(f, pos, P, cfg, s, ws));
    return eval_gather_ws(f, pos, P, u, grad, cfg, s, ws);
}

bsi_status eval_run(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                    const bsi_eval_config& cfg, hipStream_t s) {
    if (P == 0) return BSI_OK;
    void* ws = nullptr;
    const size_t need = eval_ws_bytes(f, P, cfg);
    if (need) BSI_TRY(get_workspace(f->ctx->eval_ws, s, need, &ws));
    return eval_run_ws(f, pos, P, u, grad, cfg, s, ws);
}

bsi_status debug_cells_run(bsi_field* f, const double* pos, int64_t P, int32_t* cell, double* t,
                           hipStream_t s) {
    if (P == 0) return BSI_OK;
    const CellArgs ca = cell_args(f, pos, P);
    hipLaunchKernelGGL(k_debug_cells, dim3(unsigned((P + 255) / 256)), dim3(256), 0, s, ca, cell, t);
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

bsi_status debug_bins_run(bsi_field* f, const double* pos, int64_t P, int tile, uint32_t* hist, uint32_t* offs,
                          uint32_t* perm, double* pos_sorted, hipStream_t s) {
    const size_t nb = bin_bucket_count(f, tile) + 1;
    if (P == 0) {
        BSI_HIP(hipMemsetAsync(hist, 0, nb * sizeof(uint32_t), s));
        BSI_HIP(hipMemsetAsync(offs, 0, nb * sizeof(uint32_t), s));
        return BSI_OK;
    }
    const BinLayout l = bin_layout(f, P, tile);
    void* ws = nullptr;
    BSI_TRY(get_workspace(f->ctx->eval_ws, s, l.bytes, &ws));
    char* w = static_cast<char*>(ws);
    BSI_TRY(bin_run(f, pos, P, tile, w + l.grp, reinterpret_cast<uint32_t*>(w + l.perm),
                    reinterpret_cast<double*>(w + l.pos), reinterpret_cast<uint32_t*>(w + l.hist),
                    reinterpret_cast<uint32_t*>(w + l.offs), s));
    BSI_HIP(hipMemcpyAsync(hist, w + l.hist, nb * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    BSI_HIP(hipMemcpyAsync(offs, w + l.offs, nb * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    BSI_HIP(hipMemcpyAsync(perm, w + l.perm, size_t(P) * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    BSI_HIP(hipMemcpyAsync(pos_sorted, w + l.pos, size_t(P) * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    return BSI_OK;
}

}  // namespace bsi
