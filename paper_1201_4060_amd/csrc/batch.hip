// Batched evaluation: many fields with uneven particle sets evaluated by one
// persistent gather launch, optionally captured once into a HIP graph and
// replayed.  The per-particle arithmetic is the single-field one
// (gather.hpp), so every item's result is bitwise the result of bsi_eval_ex
// with the same configuration.
//
// Plan (host, at creation): items are laid end to end in one particle index
// space and one bucket index space.  Each item is binned by the Morton tile of
// its own sort granularity; the tuned (or given) configuration decides per
// item whether its particles are gathered tile by tile from LDS (tiles of 8^3
// cells) or one lane per particle from global memory.
//
// Device work (one stream, no host synchronisation in between):
//   fill        zero the work counters
//   grouping    cell and Morton bucket of every particle (all items at once),
//               grouped by bucket without global atomics (gather.hpp): bucket
//               table, binned permutation and binned copy of the positions
//   compact     list of the non-empty buckets of the tiled items, one list
//               per (order, components) class
//   gather      per class present: a persistent grid of resident one-wavefront
//               workgroups striding over the class's non-empty tiles, and a
//               plain grid with one wavefront per group of 64 consecutive
//               binned particles of the class's direct items.  One kernel per
//               class and path keeps each kernel's registers and LDS to what
//               its own bodies need.
#include <algorithm>
#include <string>
#include <vector>

#include "gather.hpp"

namespace bsi {

namespace {

constexpr int BATCH_B = 64;        // threads per workgroup of the persistent tile gather
constexpr int UNIT = 64;           // particles per direct unit (one wavefront)
constexpr int DIRECT_B = 256;      // threads per workgroup of the direct gather
constexpr int BLK = 256;           // threads per workgroup of the binning kernels
constexpr int NCLASS = 4;          // (order, components) classes: (4,1) (4,3) (6,1) (6,3)

constexpr int class_of(int N, int C) { return (N == 6 ? 2 : 0) + (C == 3 ? 1 : 0); }
enum : int32_t { MODE_DIRECT = 0, MODE_TILE8 = 2 };

struct BatchItem {
    GatherArgs ga;       // hist/offs at the item's buckets; perm/pos_sorted are the batch-wide arrays
    int32_t N, C, mode, tile;
    int32_t cls;         // class_of(N, C)
    uint32_t pbase;      // first particle slot of the item in the batch
    uint32_t bbase;      // first bucket of the item in the batch
    uint32_t nb;         // buckets of the item, the non-finite bucket included
    uint32_t pblk;       // first binning workgroup of the item
    uint32_t bblk;       // first compaction workgroup of the item (tiled items)
    uint32_t ubase;      // first direct unit of the item (direct items; units are grouped by class)
    uint32_t cbase;      // first coarse grouping range of the item
    int32_t cshift;      // item bucket b lies in coarse range cbase + (b >> cshift)
};

struct BatchArgs {
    const BatchItem* items;
    const uint16_t* pblock_item;  // item of each binning workgroup
    const uint16_t* bblock_item;  // item of each compaction workgroup
    const uint16_t* dunit_item;   // item of each direct unit
    uint32_t* hist;
    uint32_t* offs;
    uint32_t* perm;
    double* pos_sorted;
    const uint32_t* cstart;       // first bucket of every coarse grouping range (+ end)
    uint2* tile_list;             // (item, bucket) of every non-empty tile, class by class
    uint32_t* ctr;                // [1 + class] non-empty tiles of the class ([0] unused)
    uint32_t lbase[NCLASS];       // first tile-list slot of each class
};

// cell -> item-local Morton bucket, or the item's non-finite bucket
__device__ __forceinline__ uint32_t item_bucket(const BatchItem& it, const double* x) {
    const int n[3] = {it.ga.n0, it.ga.n1, it.ga.n2};
    const double ih[3] = {it.ga.ih0, it.ga.ih1, it.ga.ih2};
    int c[3];
    double t[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) ok = cell_of(x[d], ih[d], n[d], c[d], t[d]) && ok;
    if (!ok) return it.nb - 1;
    const uint32_t T = uint32_t(it.tile);
    return (spread3(uint32_t(c[0]) / T) << 2) | (spread3(uint32_t(c[1]) / T) << 1) |
           spread3(uint32_t(c[2]) / T);
}

// Grouping slots of a batch: item i owns the slots [pblk * BLK, (pblk +
// ceil(P / BLK)) * BLK), slot pblk * BLK + p holding its particle p; the
// slots past P are padding.
struct BatchSlots {
    const BatchItem* items;
    const uint16_t* pblock_item;
    __device__ __forceinline__ const BatchItem& item_of(long i, long& p) const {
        const BatchItem& it = items[pblock_item[i / BLK]];
        p = i - long(it.pblk) * BLK;
        return it;
    }
    __device__ __forceinline__ bool key(long i, uint32_t& k, uint32_t& c) const {
        long p;
        const BatchItem& it = item_of(i, p);
        if (p >= it.ga.P) return false;
        const double x[3] = {it.ga.pos[3 * p], it.ga.pos[3 * p + 1], it.ga.pos[3 * p + 2]};
        const uint32_t lk = item_bucket(it, x);
        k = it.bbase + lk;
        c = it.cbase + (lk >> it.cshift);
        return true;
    }
    __device__ __forceinline__ uint32_t coarse(long i, uint32_t k) const {
        long p;
        const BatchItem& it = item_of(i, p);
        return it.cbase + ((k - it.bbase) >> it.cshift);
    }
    __device__ __forceinline__ void fetch(long i, uint32_t& local, double* x) const {
        long p;
        const BatchItem& it = item_of(i, p);
        local = uint32_t(p);
        x[0] = it.ga.pos[3 * p];
        x[1] = it.ga.pos[3 * p + 1];
        x[2] = it.ga.pos[3 * p + 2];
    }
};

// Coarse ranges of a batch: range c holds the batch buckets [cstart[c],
// cstart[c + 1]).
struct TableCoarse {
    const uint32_t* cstart;
    __device__ __forceinline__ void range(uint32_t c, uint32_t& lo, uint32_t& hi) const {
        lo = cstart[c];
        hi = cstart[c + 1];
    }
};

__global__ __launch_bounds__(BLK) void k_batch_compact(BatchArgs b) {
    const uint32_t item = b.bblock_item[blockIdx.x];
    const BatchItem& it = b.items[item];
    const uint32_t k = (blockIdx.x - it.bblk) * BLK + threadIdx.x;
    if (k >= it.nb) return;
    if (b.hist[it.bbase + k] != 0u)
        b.tile_list[b.lbase[it.cls] + atomicAdd(&b.ctr[1 + it.cls], 1u)] = make_uint2(item, k);
}

template <int N, typename CT, int C, int T>
constexpr bool batch_tile_ok() {
    return TileGeom<N, CT, C, T>::BYTES <= 65536 && TileGeom<N, CT, C, T>::ALIGNED &&
           TileGeom<N, CT, C, T>::SLOTS < 3072;
}

// Tiles of class (N, C): workgroup g takes the class's tiles g, g + G, g + 2G,
// ... (G = grid size); the tile index is the same in every lane, so the loop
// is scalar and every wavefront of the workgroup meets the same barriers.
template <typename CT, bool GRAD, int N, int C>
__global__ __launch_bounds__(BATCH_B) void k_batch_tiles(BatchArgs b) {
    if constexpr (batch_tile_ok<N, CT, C, 8>()) {
        extern __shared__ u32x4 lds[];
        constexpr int cls = class_of(N, C);
        const uint32_t ntile = __builtin_amdgcn_readfirstlane(b.ctr[1 + cls]);
        const uint2* list = b.tile_list + b.lbase[cls];
        for (uint32_t u = blockIdx.x; u < ntile; u += gridDim.x) {
            const uint2 e = list[u];
            const uint32_t item = __builtin_amdgcn_readfirstlane(e.x);
            const uint32_t bucket = __builtin_amdgcn_readfirstlane(e.y);
            tile_eval<N, CT, C, GRAD, 8, BATCH_B>(b.items[item].ga, bucket, lds);
        }
    }
}

// Direct units [d0, d1) of class (N, C), one wavefront each: lane l of unit d
// takes binned particle (d - ubase) * UNIT + l of the unit's item.  The
// kernel has no barrier, so lanes without a particle leave at once.
template <typename CT, bool GRAD, int N, int C>
__global__ __launch_bounds__(DIRECT_B) void k_batch_direct(BatchArgs b, uint32_t d0, uint32_t d1) {
    const uint32_t d = d0 + blockIdx.x * (DIRECT_B / UNIT) + threadIdx.x / UNIT;
    if (d >= d1) return;
    const uint32_t item = __builtin_amdgcn_readfirstlane(uint32_t(b.dunit_item[d]));
    const BatchItem& it = b.items[item];
    const long r = long(d - it.ubase) * UNIT + (threadIdx.x % UNIT);
    if (r >= it.ga.P) return;
    direct_eval<N, CT, C, GRAD>(it.ga, long(it.pbase) + r);
}

// f(CT{}, GRAD, N, C) with the launch's types as compile-time constants.
template <typename F>
void with_class(int coef, bool grad, int cls, F&& f) {
    auto by_class = [&](auto ct, auto g) {
        using I1 = std::integral_constant<int, 1>;
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        using I6 = std::integral_constant<int, 6>;
        switch (cls) {
            case 0: f(ct, g, I4{}, I1{}); break;
            case 1: f(ct, g, I4{}, I3{}); break;
            case 2: f(ct, g, I6{}, I1{}); break;
            default: f(ct, g, I6{}, I3{}); break;
        }
    };
    auto by_grad = [&](auto ct) {
        if (grad) by_class(ct, std::true_type{});
        else by_class(ct, std::false_type{});
    };
    if (coef == BSI_F64) by_grad(double{});
    else if (coef == BSI_F32) by_grad(float{});
    else by_grad(uint16_t{});
}

template <typename CT>
bool tile_supported_batch(int N, int C, int T) {
    if (T != 4 && T != 8) return false;
    if (N == 4) {
        if (C == 1) return T == 4 ? batch_tile_ok<4, CT, 1, 4>() : batch_tile_ok<4, CT, 1, 8>();
        return T == 4 ? batch_tile_ok<4, CT, 3, 4>() : batch_tile_ok<4, CT, 3, 8>();
    }
    if (C == 1) return T == 4 ? batch_tile_ok<6, CT, 1, 4>() : batch_tile_ok<6, CT, 1, 8>();
    return T == 4 ? batch_tile_ok<6, CT, 3, 4>() : batch_tile_ok<6, CT, 3, 8>();
}

bool batch_tile_supported(int coef, int N, int C, int T) {
    if (coef == BSI_F64) return tile_supported_batch<double>(N, C, T);
    if (coef == BSI_F32) return tile_supported_batch<float>(N, C, T);
    return tile_supported_batch<uint16_t>(N, C, T);
}

template <typename CT>
int tile_lds_ct(int N, int C, int T) {
    auto one = [&](auto n_, auto c_, auto t_) -> int {
        constexpr int n = decltype(n_)::value, c = decltype(c_)::value, t = decltype(t_)::value;
        return tile_lds_bytes<n, CT, c, t, BATCH_B>();
    };
    using I4 = std::integral_constant<int, 4>;
    using I6 = std::integral_constant<int, 6>;
    using I1 = std::integral_constant<int, 1>;
    using I3 = std::integral_constant<int, 3>;
    using I8 = std::integral_constant<int, 8>;
    if (N == 4) {
        if (C == 1) return T == 4 ? one(I4{}, I1{}, I4{}) : one(I4{}, I1{}, I8{});
        return T == 4 ? one(I4{}, I3{}, I4{}) : one(I4{}, I3{}, I8{});
    }
    if (C == 1) return T == 4 ? one(I6{}, I1{}, I4{}) : one(I6{}, I1{}, I8{});
    return T == 4 ? one(I6{}, I3{}, I4{}) : one(I6{}, I3{}, I8{});
}

int batch_tile_lds(int coef, int N, int C, int T) {
    if (coef == BSI_F64) return tile_lds_ct<double>(N, C, T);
    if (coef == BSI_F32) return tile_lds_ct<float>(N, C, T);
    return tile_lds_ct<uint16_t>(N, C, T);
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

}  // namespace bsi

using namespace bsi;

struct bsi_batch {
    bsi_ctx* ctx = nullptr;
    std::vector<bsi_eval_config> cfgs;   // per item, as planned
    int coef = BSI_F32;
    bool grad = true;
    int nitems = 0;                      // items with P > 0
    uint64_t Ptot = 0, Btot = 0;
    uint32_t nbblocks = 0;
    uint32_t dbeg[NCLASS] = {}, dend[NCLASS] = {};  // direct units of each class
    uint32_t tbound[NCLASS] = {};   // buckets of the class's tiled items (bound on its tiles)
    unsigned tgrid[NCLASS] = {};    // persistent tile grid of each class
    size_t tlds[NCLASS] = {};       // LDS of the class's tile workgroups
    GrpPlan grp;                         // grouping of the particle slots by bucket
    GrpBuffers gbuf{};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    BatchArgs args{};
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace bsi {

// Plan choice of one item from a configuration: a tiled configuration keeps
// the tiled gather, with the batch kernel's 8^3-cell tiles when the class has
// them; anything else is gathered one lane per particle, binned with the
// configuration's tile.
static void item_mode(const bsi_field* f, const bsi_eval_config& c, int* mode, int* tile) {
    const int nmax = std::max(f->n[0], std::max(f->n[1], f->n[2]));
    const int tmin = (nmax + 255) / 256;  // at most 2^24 buckets
    if (c.variant == 0 && c.sort_tile > 0 && 8 >= tmin && batch_tile_supported(f->desc.coef, f->N, f->C, 8)) {
        *mode = MODE_TILE8;
        *tile = 8;
        return;
    }
    *mode = MODE_DIRECT;
    *tile = std::max(c.sort_tile > 0 ? c.sort_tile : 8, tmin);
}

size_t bin_bucket_count(const bsi_field* f, int tile);  // eval.hip

static bsi_status enqueue(bsi_batch* b, hipStream_t s) {
    bsi_ctx* ctx = b->ctx;
    if (b->nitems == 0) return BSI_OK;
    const BatchArgs& a = b->args;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, a.ctr, long(1 + NCLASS), 0u);
    {
        StageTimer tm(ctx, "batch_bin", s);
        const BatchSlots slots{a.items, a.pblock_item};
        grp_count(slots, b->grp, b->gbuf, s);
        grp_scan(b->grp, b->gbuf, s);
        grp_scatter(slots, TableCoarse{a.cstart}, b->grp, b->gbuf, a.hist, a.offs, a.perm, a.pos_sorted, s);
        if (b->nbblocks) hipLaunchKernelGGL(k_batch_compact, dim3(b->nbblocks), dim3(BLK), 0, s, a);
    }
    {
        StageTimer tm(ctx, "batch_gather", s);
        for (int cls = 0; cls < NCLASS; ++cls) {
            const unsigned tg = b->tgrid[cls];
            const size_t tl = b->tlds[cls];
            const uint32_t d0 = b->dbeg[cls], d1 = b->dend[cls];
            const unsigned dg = unsigned((d1 - d0 + DIRECT_B / UNIT - 1) / (DIRECT_B / UNIT));
            with_class(b->coef, b->grad, cls, [&](auto ct, auto g, auto n, auto c) {
                using CT = decltype(ct);
                constexpr bool G = decltype(g)::value;
                constexpr int N = decltype(n)::value, C = decltype(c)::value;
                if (tg) hipLaunchKernelGGL((k_batch_tiles<CT, G, N, C>), dim3(tg), dim3(BATCH_B), tl, s, a);
                if (dg) hipLaunchKernelGGL((k_batch_direct<CT, G, N, C>), dim3(dg), dim3(DIRECT_B), 0, s, a, d0, d1);
            });
        }
    }
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

}  // namespace bsi

extern "C" {

bsi_status bsi_batch_create(bsi_ctx* ctx, const bsi_eval_item* items, int32_t count,
                            const bsi_eval_config* cfgs, bsi_batch** out) {
    clear_error();
    BSI_CHECK(ctx && out, BSI_E_INVAL, "NULL argument");
    *out = nullptr;
    BSI_CHECK(count >= 1 && count <= 65535, BSI_E_INVAL, "count must be in [1, 65535]");
    BSI_CHECK(items != nullptr, BSI_E_INVAL, "items is NULL");
    const bsi_field* f0 = items[0].field;
    BSI_CHECK(f0 != nullptr, BSI_E_INVAL, "item 0 has no field");
    const int coef = f0->desc.coef;
    // grad presence is decided on the items with particles (empty tensors may
    // come with NULL pointers)
    bool grad = items[0].grad != nullptr;
    for (int i = 0; i < count; ++i)
        if (items[i].P > 0) {
            grad = items[i].grad != nullptr;
            break;
        }
    uint64_t Ptot = 0;
    for (int i = 0; i < count; ++i) {
        const bsi_eval_item& it = items[i];
        const std::string tag = "item " + std::to_string(i) + ": ";
        BSI_CHECK(it.field != nullptr, BSI_E_INVAL, tag + "field is NULL");
        BSI_CHECK(it.field->ctx == ctx, BSI_E_INVAL, tag + "field belongs to another context");
        BSI_CHECK(it.field->basis == BSI_BASIS_BSPLINE && (it.field->N == 4 || it.field->N == 6),
                  BSI_E_UNSUPPORTED, tag + "batches hold B-spline fields of orders 4 and 6");
        BSI_CHECK(it.field->desc.coef == coef, BSI_E_INVAL,
                  tag + "a batch holds fields of one coefficient type");
        BSI_CHECK(it.P >= 0 && it.P < (int64_t(1) << 31), BSI_E_INVAL, tag + "P must be in [0, 2^31)");
        if (it.P == 0) continue;
        BSI_CHECK((it.grad != nullptr) == grad, BSI_E_INVAL,
                  tag + "grad must be given for every item of a batch or for none");
        BSI_TRY(check_device_ptr_ex(it.pos, (tag + "pos").c_str()));
        BSI_TRY(check_device_ptr_ex(it.u, (tag + "u").c_str()));
        if (grad) BSI_TRY(check_device_ptr_ex(it.grad, (tag + "grad").c_str()));
        if (cfgs) {
            const bsi_eval_config& c = cfgs[i];
            BSI_CHECK(c.sort_tile >= 0 && c.sort_tile <= 1024, BSI_E_INVAL, tag + "sort_tile out of range");
        }
        Ptot += uint64_t(it.P);
    }
    BSI_CHECK(Ptot < (uint64_t(1) << 31), BSI_E_INVAL, "a batch holds fewer than 2^31 particles");
    BSI_HIP(hipSetDevice(ctx->device));

    auto* b = new (std::nothrow) bsi_batch();
    BSI_CHECK(b != nullptr, BSI_E_NOMEM, "host allocation failed");
    b->ctx = ctx;
    b->coef = coef;
    b->grad = grad;
    b->cfgs.resize(count);
    std::vector<BatchItem> hi;
    std::vector<uint16_t> pblock, bblock, dunit_cls[NCLASS];
    uint64_t Btot = 0, pbase = 0;
    for (int i = 0; i < count; ++i) {
        const bsi_eval_item& it = items[i];
        bsi_field* f = it.field;
        bsi_eval_config c{};
        if (cfgs) c = cfgs[i];
        else if (bsi_status st = lookup_config(ctx, f, it.P, &c); st != BSI_OK) {
            delete b;
            return st;
        }
        b->cfgs[i] = c;
        if (it.P == 0) continue;
        int mode = 0, tile = 0;
        item_mode(f, c, &mode, &tile);
        b->cfgs[i].variant = mode == MODE_DIRECT ? 1 : 0;
        b->cfgs[i].sort_tile = tile;
        BatchItem x{};
        GatherArgs& g = x.ga;
        g.grid = f->grid;
        g.pos = it.pos;
        g.u = it.u;
        g.grad = it.grad;
        g.nonfinite = f->counters;
        g.P = long(it.P);
        g.n0 = f->n[0];
        g.n1 = f->n[1];
        g.n2 = f->n[2];
        g.P1 = f->P[1];
        g.P2 = f->P[2];
        g.pitch2 = f->pitch2;
        g.ih0 = f->inv_h[0];
        g.ih1 = f->inv_h[1];
        g.ih2 = f->inv_h[2];
        g.xcd_remap = 0;
        g.tiles_per_group = 1;
        g.basis = BSI_BASIS_BSPLINE;
        g.cs = 1;
        const size_t nbf = bin_bucket_count(f, tile);
        g.nbuckets_finite = uint32_t(nbf);
        x.N = f->N;
        x.C = f->C;
        x.cls = class_of(f->N, f->C);
        x.mode = mode;
        x.tile = tile;
        x.pbase = uint32_t(pbase);
        x.bbase = uint32_t(Btot);
        x.nb = uint32_t(nbf + 1);
        x.pblk = uint32_t(pblock.size());
        const uint16_t id = uint16_t(hi.size());
        pblock.insert(pblock.end(), size_t((it.P + BLK - 1) / BLK), id);
        if (mode == MODE_DIRECT) {
            std::vector<uint16_t>& du = dunit_cls[x.cls];
            x.ubase = uint32_t(du.size());  // class-local until the classes are laid end to end
            du.insert(du.end(), size_t((it.P + UNIT - 1) / UNIT), id);
        } else {
            x.bblk = uint32_t(bblock.size());
            bblock.insert(bblock.end(), size_t((x.nb + BLK - 1) / BLK), id);
            b->tbound[x.cls] += x.nb;
            b->tlds[x.cls] = size_t(batch_tile_lds(coef, f->N, f->C, tile));
        }
        hi.push_back(x);
        pbase += uint64_t(it.P);
        Btot += nbf + 1;
    }
    // coarse grouping ranges: per item about `target` particles each; the
    // target doubles until all of them fit the grouping's LDS table
    std::vector<uint32_t> cstart;
    for (uint64_t target = GRP_TARGET;; target *= 2) {
        uint64_t nc = 0;
        for (auto& x : hi) {
            x.cshift = grp_shift(x.nb, long(x.ga.P), target);
            x.cbase = uint32_t(nc);
            nc += (uint64_t(x.nb) + (uint64_t(1) << x.cshift) - 1) >> x.cshift;
        }
        if (nc <= GRP_COARSE_MAX) break;
        if (target > (uint64_t(1) << 40)) {
            delete b;
            set_error("too many buckets in one batch; use coarser sort tiles");
            return BSI_E_INVAL;
        }
    }
    // direct units class by class, tile-list slots class by class
    std::vector<uint16_t> dunit;
    for (int c = 0; c < NCLASS; ++c) {
        b->dbeg[c] = uint32_t(dunit.size());
        dunit.insert(dunit.end(), dunit_cls[c].begin(), dunit_cls[c].end());
        b->dend[c] = uint32_t(dunit.size());
    }
    for (auto& x : hi)
        if (x.mode == MODE_DIRECT) x.ubase += b->dbeg[x.cls];
    uint32_t lbase[NCLASS];
    {
        uint64_t l = 0;
        for (int c = 0; c < NCLASS; ++c) {
            lbase[c] = uint32_t(l);
            l += b->tbound[c];
        }
    }
    uint32_t fine_max = 1;
    for (const auto& x : hi) {
        for (uint64_t lo = 0; lo < x.nb; lo += uint64_t(1) << x.cshift) cstart.push_back(uint32_t(x.bbase + lo));
        fine_max = std::max(fine_max, std::min<uint32_t>(x.nb, uint32_t(1) << x.cshift));
    }
    cstart.push_back(uint32_t(Btot));
    if (Btot >= (uint64_t(1) << 32)) {
        delete b;
        set_error("too many buckets in one batch; use coarser sort tiles");
        return BSI_E_INVAL;
    }
    b->grp = grp_plan(long(pblock.size()) * BLK, uint32_t(pbase), uint32_t(Btot), uint32_t(cstart.size() - 1),
                      fine_max);
    b->nitems = int(hi.size());
    b->Ptot = pbase;
    b->Btot = Btot;
    b->nbblocks = uint32_t(bblock.size());
    if (b->nitems == 0) {
        *out = b;
        return BSI_OK;
    }
    // workspace: tables, bucket table (counts, offsets), grouping scratch,
    // perm, binned positions, tile list, counters
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_items = take(hi.size() * sizeof(BatchItem));
    const size_t o_pblock = take(pblock.size() * sizeof(uint16_t));
    const size_t o_bblock = take(std::max<size_t>(bblock.size(), 1) * sizeof(uint16_t));
    const size_t o_dunit = take(std::max<size_t>(dunit.size(), 1) * sizeof(uint16_t));
    const size_t o_hist = take(Btot * sizeof(uint32_t));
    const size_t o_offs = take(Btot * sizeof(uint32_t));
    const size_t o_grp = take(grp_scratch_words(b->grp) * sizeof(uint32_t));
    const size_t o_cstart = take(cstart.size() * sizeof(uint32_t));
    const size_t o_perm = take(pbase * sizeof(uint32_t));
    const size_t o_pos = take(3 * pbase * sizeof(double));
    const size_t o_list = take(std::max<uint64_t>(Btot, 1) * sizeof(uint2));
    const size_t o_ctr = take((1 + NCLASS) * sizeof(uint32_t));
    b->ws_bytes = off;
    if (hipMalloc(&b->ws, off) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        set_error("batch workspace allocation of " + std::to_string(off) + " bytes failed");
        return BSI_E_NOMEM;
    }
    char* base = static_cast<char*>(b->ws);
    BatchArgs& a = b->args;
    a.items = reinterpret_cast<const BatchItem*>(base + o_items);
    a.pblock_item = reinterpret_cast<const uint16_t*>(base + o_pblock);
    a.bblock_item = reinterpret_cast<const uint16_t*>(base + o_bblock);
    a.dunit_item = reinterpret_cast<const uint16_t*>(base + o_dunit);
    a.hist = reinterpret_cast<uint32_t*>(base + o_hist);
    a.offs = reinterpret_cast<uint32_t*>(base + o_offs);
    b->gbuf = grp_buffers(b->grp, reinterpret_cast<uint32_t*>(base + o_grp));
    a.cstart = reinterpret_cast<const uint32_t*>(base + o_cstart);
    a.perm = reinterpret_cast<uint32_t*>(base + o_perm);
    a.pos_sorted = reinterpret_cast<double*>(base + o_pos);
    a.tile_list = reinterpret_cast<uint2*>(base + o_list);
    a.ctr = reinterpret_cast<uint32_t*>(base + o_ctr);
    for (int c = 0; c < NCLASS; ++c) a.lbase[c] = lbase[c];
    for (auto& x : hi) {
        x.ga.hist = a.hist + x.bbase;
        x.ga.offs = a.offs + x.bbase;
        x.ga.perm = a.perm;
        x.ga.pos_sorted = a.pos_sorted;
    }
    bsi_status st = BSI_OK;
    auto up = [&](size_t o, const void* src, size_t bytes) {
        if (st == BSI_OK && bytes && hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            set_error("upload of the batch tables failed");
            st = BSI_E_DEVICE;
        }
    };
    up(o_items, hi.data(), hi.size() * sizeof(BatchItem));
    up(o_pblock, pblock.data(), pblock.size() * sizeof(uint16_t));
    up(o_bblock, bblock.data(), bblock.size() * sizeof(uint16_t));
    up(o_dunit, dunit.data(), dunit.size() * sizeof(uint16_t));
    up(o_cstart, cstart.data(), cstart.size() * sizeof(uint32_t));
    // persistent tile grids: as many one-wavefront workgroups as stay
    // resident, at most one per bucket of the class's tiled items
    for (int c = 0; c < NCLASS && st == BSI_OK; ++c) {
        if (b->tbound[c] == 0) continue;
        int per_cu = 0;
        with_class(coef, grad, c, [&](auto ct, auto g, auto n, auto cc) {
            using CT = decltype(ct);
            constexpr bool G = decltype(g)::value;
            constexpr int N = decltype(n)::value, C = decltype(cc)::value;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, reinterpret_cast<const void*>(&k_batch_tiles<CT, G, N, C>), BATCH_B, b->tlds[c]) !=
                hipSuccess) {
                (void)hipGetLastError();
                per_cu = 0;
            }
        });
        per_cu = std::max(1, std::min(per_cu, 32));
        b->tgrid[c] = unsigned(std::min<uint64_t>(uint64_t(per_cu) * ctx->num_cus, b->tbound[c]));
    }
    if (st != BSI_OK) {
        (void)hipFree(b->ws);
        delete b;
        return st;
    }
    *out = b;
    return BSI_OK;
}

bsi_status bsi_batch_run(bsi_batch* b, int32_t use_graph, void* stream) {
    clear_error();
    BSI_CHECK(b != nullptr, BSI_E_INVAL, "batch is NULL");
    BSI_HIP(hipSetDevice(b->ctx->device));
    hipStream_t s = pick_stream(b->ctx, stream);
    if (!use_graph) return enqueue(b, s);
    if (!b->exec) {
        // capture once on a private stream; the graph is then launched on `s`
        if (!b->cap_stream) BSI_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        BSI_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        const bsi_status st = enqueue(b, b->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (st != BSI_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        BSI_CHECK(e == hipSuccess && g, BSI_E_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
        b->graph = g;
        BSI_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    StageTimer tm(b->ctx, "batch_graph", s);
    BSI_HIP(hipGraphLaunch(b->exec, s));
    return BSI_OK;
}

bsi_status bsi_batch_item_config(const bsi_batch* b, int32_t item, bsi_eval_config* cfg) {
    clear_error();
    BSI_CHECK(b && cfg, BSI_E_INVAL, "NULL argument");
    BSI_CHECK(item >= 0 && item < int32_t(b->cfgs.size()), BSI_E_INVAL, "item out of range");
    *cfg = b->cfgs[item];
    return BSI_OK;
}

size_t bsi_batch_bytes(const bsi_batch* b) { return b ? b->ws_bytes : 0; }

void bsi_batch_destroy(bsi_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->ws) (void)hipFree(b->ws);
    delete b;
}

bsi_status bsi_eval_batch(bsi_ctx* ctx, const bsi_eval_item* items, int32_t count, void* stream) {
    bsi_batch* b = nullptr;
    BSI_TRY(bsi_batch_create(ctx, items, count, nullptr, &b));
    hipStream_t s = pick_stream(ctx, stream);
    bsi_status st = bsi_batch_run(b, 0, s);
    if (st == BSI_OK && hipStreamSynchronize(s) != hipSuccess) {
        set_error(std::string("batch failed: ") + hipGetErrorString(hipGetLastError()));
        st = BSI_E_DEVICE;
    }
    bsi_batch_destroy(b);
    return st;
}

}  // extern "C"
