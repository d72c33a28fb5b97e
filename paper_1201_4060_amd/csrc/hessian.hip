// Second derivatives of the interpolant, with u and grad u.
//
// Section 2: the l-th derivative of the interpolant on a cell uses the matrix
// M^(l) = M D^l; here l = 2 gives the weights w''_j(t).  In three dimensions
// (Section 3) the mixed derivative d2/dx_i dx_j takes the first-derivative
// weights on axes i and j, and d2/dx_i^2 the second-derivative weights on
// axis i; every factor carries the chain factor n/L of its axis.  The
// particles are binned as for the evaluation (Morton tiles of 8^3 cells) and
// gathered from an LDS copy of each tile's block of the grid (or, for classes
// without a tiled body, one lane per particle straight from the grid), the
// contraction reducing axis 2 first, then axis 1, then axis 0 (the Table 1
// idea), with six per-plane partial sums per component instead of three.
//
// Output per particle p and component c: u[p][c], grad[p][c][d] and
// hess[p][c][m] = d2 u_c / dx_i dx_j for (i, j) = (0,0), (0,1), (0,2), (1,1),
// (1,2), (2,2) in that order.
#include <algorithm>

#include "gather.hpp"

namespace bsi {

namespace {

constexpr int HESS_B = 256;

// M^(2)[r][c] = (c+1)(c+2) M[r][c+2] (M D^2, Section 2), at compile time.
template <int N>
struct BSpline2 {
    double M2[N][N];
    constexpr BSpline2() : M2{} {
        for (int r = 0; r < N; ++r)
            for (int c = 0; c < N; ++c)
                M2[r][c] = (c + 2 < N) ? double((c + 1) * (c + 2) * bspline_numer(N, r, c + 2)) /
                                             double(fact_ll(N - 1))
                                       : 0.0;
    }
};

// w''_j(t) = sum_i M^(2)[j][i] t^i (Horner)
template <int N, typename AT>
__device__ __forceinline__ void bspline_weights2(AT t, AT* wdd) {
    constexpr BSpline2<N> B{};
#pragma unroll
    for (int j = 0; j < N; ++j) {
        AT acc = AT(B.M2[j][N - 3]);
#pragma unroll
        for (int i = N - 4; i >= 0; --i) acc = acc * t + AT(B.M2[j][i]);
        wdd[j] = acc;
    }
}

struct HessArgs {
    const void* grid;
    const double* pos_sorted;  // positions in binned order
    const uint32_t* perm;      // particle of every binned slot
    const uint32_t* hist;      // particles per Morton tile (tiled kernel)
    const uint32_t* offs;      // first binned slot per Morton tile (tiled kernel)
    uint32_t nbf;              // finite tiles; tile nbf holds the particles without a cell
    long P;
    int n0, n1, n2, P1;
    long pitch2;
    double ih0, ih1, ih2;
    void* u;
    void* grad;  // or nullptr
    void* hess;
    unsigned long long* nonfinite;
    const u32x4* items;        // work items (bucket, first slot, count) in bucket order (tiled kernel)
    uint32_t* ctl;             // item count and per-range counters (tiled kernel)
};

// One lane per binned slot j; results are written at the particle's index.
template <int N, typename CT, int C>
__global__ __launch_bounds__(HESS_B) void k_gather_hess(HessArgs a) {
    using AT = typename Acc<CT>::type;
    const long j = long(blockIdx.x) * HESS_B + threadIdx.x;
    if (j >= a.P) return;
    const long p = long(a.perm[j]);
    const double x[3] = {a.pos_sorted[3 * j], a.pos_sorted[3 * j + 1], a.pos_sorted[3 * j + 2]};
    const int n[3] = {a.n0, a.n1, a.n2};
    const double ih[3] = {a.ih0, a.ih1, a.ih2};
    int cell[3];
    double t[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) ok = cell_of(x[d], ih[d], n[d], cell[d], t[d]) && ok;
    AT* u = static_cast<AT*>(a.u) + p * C;
    AT* g = a.grad ? static_cast<AT*>(a.grad) + p * C * 3 : nullptr;
    AT* h = static_cast<AT*>(a.hess) + p * C * 6;
    if (!ok) {
        const AT nan = AT(__builtin_nan(""));
        for (int c = 0; c < C; ++c) u[c] = nan;
        if (g)
            for (int c = 0; c < 3 * C; ++c) g[c] = nan;
        for (int c = 0; c < 6 * C; ++c) h[c] = nan;
        atomicAdd(a.nonfinite, 1ull);
        return;
    }
    AT w[3][N], wd[3][N], wdd[3][N];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        bspline_weights<N, AT>(AT(t[d]), w[d], wd[d]);
        bspline_weights2<N, AT>(AT(t[d]), wdd[d]);
        const AT s = AT(ih[d]);
        const AT s2 = AT(ih[d] * ih[d]);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            wd[d][k] *= s;
            wdd[d][k] *= s2;
        }
    }
    const CT* base = static_cast<const CT*>(a.grid) + (long(cell[0]) * a.P1 + cell[1]) * a.pitch2 +
                     long(cell[2]) * C;
    const long rowA = long(a.P1) * a.pitch2;
    const long rowB = a.pitch2;
    AT U[C], G0[C], G1[C], G2[C], H00[C], H01[C], H02[C], H11[C], H12[C], H22[C];
#pragma unroll
    for (int c = 0; c < C; ++c)
        U[c] = G0[c] = G1[c] = G2[c] = H00[c] = H01[c] = H02[c] = H11[c] = H12[c] = H22[c] = AT(0);
#pragma unroll 1
    for (int ia = 0; ia < N; ++ia) {
        AT v[C], v1[C], v2[C], v11[C], v12[C], v22[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = v1[c] = v2[c] = v11[c] = v12[c] = v22[c] = AT(0);
#pragma unroll
        for (int ib = 0; ib < N; ++ib) {
            const CT* r = base + ia * rowA + ib * rowB;
            AT tr[C], trd[C], trdd[C];
#pragma unroll
            for (int c = 0; c < C; ++c) tr[c] = trd[c] = trdd[c] = AT(0);
#pragma unroll
            for (int e = 0; e < N; ++e) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const AT val = widen<CT, AT>(r[e * C + c]);
                    tr[c] += w[2][e] * val;
                    trd[c] += wd[2][e] * val;
                    trdd[c] += wdd[2][e] * val;
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                v[c] += w[1][ib] * tr[c];
                v1[c] += wd[1][ib] * tr[c];
                v2[c] += w[1][ib] * trd[c];
                v11[c] += wdd[1][ib] * tr[c];
                v12[c] += wd[1][ib] * trd[c];
                v22[c] += w[1][ib] * trdd[c];
            }
        }
        // the axis-0 weights of plane ia, picked without dynamic indexing
        AT w0 = w[0][0], wd0 = wd[0][0], wdd0 = wdd[0][0];
#pragma unroll
        for (int k = 1; k < N; ++k) {
            w0 = ia == k ? w[0][k] : w0;
            wd0 = ia == k ? wd[0][k] : wd0;
            wdd0 = ia == k ? wdd[0][k] : wdd0;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            U[c] += w0 * v[c];
            G0[c] += wd0 * v[c];
            G1[c] += w0 * v1[c];
            G2[c] += w0 * v2[c];
            H00[c] += wdd0 * v[c];
            H01[c] += wd0 * v1[c];
            H02[c] += wd0 * v2[c];
            H11[c] += w0 * v11[c];
            H12[c] += w0 * v12[c];
            H22[c] += w0 * v22[c];
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        u[c] = U[c];
        if (g) {
            g[3 * c + 0] = G0[c];
            g[3 * c + 1] = G1[c];
            g[3 * c + 2] = G2[c];
        }
        h[6 * c + 0] = H00[c];
        h[6 * c + 1] = H01[c];
        h[6 * c + 2] = H02[c];
        h[6 * c + 3] = H11[c];
        h[6 * c + 4] = H12[c];
        h[6 * c + 5] = H22[c];
    }
}

// Cell and weights (value, first and second derivative, chain factors
// included) of the particle at x; false when it has no cell.
template <int N, typename AT>
__device__ __forceinline__ bool hess_setup(const HessArgs& a, const double* x, int* cell, AT (*w)[N],
                                           AT (*wd)[N], AT (*wdd)[N]) {
    const int n[3] = {a.n0, a.n1, a.n2};
    const double ih[3] = {a.ih0, a.ih1, a.ih2};
    double t[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) ok = cell_of(x[d], ih[d], n[d], cell[d], t[d]) && ok;
    if (!ok) return false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        bspline_weights<N, AT>(AT(t[d]), w[d], wd[d]);
        bspline_weights2<N, AT>(AT(t[d]), wdd[d]);
        const AT s = AT(ih[d]);
        const AT s2 = AT(ih[d] * ih[d]);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            wd[d][k] *= s;
            wdd[d][k] *= s2;
        }
    }
    return true;
}

// Sums over axis-0 planes: u, the three first and six second derivatives.
template <typename AT, int C>
struct HessSums {
    AT s[10][C];
};

// Planes k = 0..NP-1 with axis-0 weights w0[k], wd0[k], wdd0[k] and rows
// row(k, ib), accumulated in plane order into out (axis 2 first, then 1).
template <int N, typename CT, typename AT, int C, int NP, typename RowFn>
__device__ __forceinline__ void hess_planes(const AT* w0, const AT* wd0, const AT* wdd0, const AT (*w)[N],
                                            const AT (*wd)[N], const AT (*wdd)[N], RowFn row,
                                            HessSums<AT, C>& out) {
#pragma unroll
    for (int m = 0; m < 10; ++m)
#pragma unroll
        for (int c = 0; c < C; ++c) out.s[m][c] = AT(0);
#pragma unroll 1
    for (int k = 0; k < NP; ++k) {
        AT a0 = w0[0], d0 = wd0[0], dd0 = wdd0[0];
#pragma unroll
        for (int q = 1; q < NP; ++q) {
            a0 = k == q ? w0[q] : a0;
            d0 = k == q ? wd0[q] : d0;
            dd0 = k == q ? wdd0[q] : dd0;
        }
        AT v[C], v1[C], v2[C], v11[C], v12[C], v22[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = v1[c] = v2[c] = v11[c] = v12[c] = v22[c] = AT(0);
#pragma unroll
        for (int ib = 0; ib < N; ++ib) {
            const CT* r = row(k, ib);
            CT raw[N * C];
            if constexpr (sizeof(CT) == 2 && (N * C) % 2 == 0) {
                // BF16 rows start on 2-byte boundaries: aligned dword reads and
                // a funnel shift by the misalignment, as in the gather
                typedef const __attribute__((address_space(3))) uint16_t lds_u16;
                typedef const __attribute__((address_space(3))) uint32_t lds_u32;
                lds_u16* lr = (lds_u16*)(r);
                const uint32_t mis = uint32_t(reinterpret_cast<uintptr_t>(lr)) & 2u;
                lds_u32* d = (lds_u32*)(lr - (mis >> 1));
                constexpr int ND = N * C / 2 + 1;
                uint32_t dw[ND];
#pragma unroll
                for (int q = 0; q < ND; ++q) dw[q] = d[q];
#pragma unroll
                for (int q = 0; q < N * C / 2; ++q) {
                    const uint32_t v = __builtin_amdgcn_alignbit(dw[q + 1], dw[q], mis * 8u);
                    raw[2 * q] = CT(v & 0xffffu);
                    raw[2 * q + 1] = CT(v >> 16);
                }
            } else {
#pragma unroll
                for (int e = 0; e < N * C; ++e) raw[e] = r[e];
            }
            AT tr[C], trd[C], trdd[C];
#pragma unroll
            for (int c = 0; c < C; ++c) tr[c] = trd[c] = trdd[c] = AT(0);
#pragma unroll
            for (int e = 0; e < N; ++e) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const AT val = widen<CT, AT>(raw[e * C + c]);
                    tr[c] += w[2][e] * val;
                    trd[c] += wd[2][e] * val;
                    trdd[c] += wdd[2][e] * val;
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                v[c] += w[1][ib] * tr[c];
                v1[c] += wd[1][ib] * tr[c];
                v2[c] += w[1][ib] * trd[c];
                v11[c] += wdd[1][ib] * tr[c];
                v12[c] += wd[1][ib] * trd[c];
                v22[c] += w[1][ib] * trdd[c];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            out.s[0][c] += a0 * v[c];
            out.s[1][c] += d0 * v[c];
            out.s[2][c] += a0 * v1[c];
            out.s[3][c] += a0 * v2[c];
            out.s[4][c] += dd0 * v[c];
            out.s[5][c] += d0 * v1[c];
            out.s[6][c] += d0 * v2[c];
            out.s[7][c] += a0 * v11[c];
            out.s[8][c] += a0 * v12[c];
            out.s[9][c] += a0 * v22[c];
        }
    }
}

// u, grad u (if requested) and hess of particle p from the two halves of the
// axis-0 sum.
template <typename AT, int C>
__device__ __forceinline__ void hess_store(const HessArgs& a, long p, const HessSums<AT, C>& lo,
                                           const HessSums<AT, C>& hi) {
    AT* u = static_cast<AT*>(a.u) + p * C;
    AT* h = static_cast<AT*>(a.hess) + p * C * 6;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        u[c] = lo.s[0][c] + hi.s[0][c];
#pragma unroll
        for (int m = 0; m < 6; ++m) h[6 * c + m] = lo.s[4 + m][c] + hi.s[4 + m][c];
    }
    if (a.grad) {
        AT* g = static_cast<AT*>(a.grad) + p * C * 3;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) g[3 * c + d] = lo.s[1 + d][c] + hi.s[1 + d][c];
    }
}

template <typename AT, int C>
__device__ __forceinline__ void hess_nan(const HessArgs& a, long p) {
    const AT nan = AT(__builtin_nan(""));
    AT* u = static_cast<AT*>(a.u) + p * C;
    AT* h = static_cast<AT*>(a.hess) + p * C * 6;
    for (int c = 0; c < C; ++c) u[c] = nan;
    for (int c = 0; c < 6 * C; ++c) h[c] = nan;
    if (a.grad) {
        AT* g = static_cast<AT*>(a.grad) + p * C * 3;
        for (int c = 0; c < 3 * C; ++c) g[c] = nan;
    }
}

constexpr int HESS_TB = 64;           // threads per workgroup of the tiled kernel
constexpr uint32_t HESS_ROUNDS = 4;   // rounds of one wavefront per work item

// The `count` binned particles from slot `start` of Morton tile `cur` (8^3
// cells), or of the bucket without a cell when `cur` == nbf, by one
// wavefront.  With `fill` the tile's (8+N-1)^3 block of the grid is first
// copied into LDS by the load unit's DMA path (else the LDS holds it from the
// previous call); then every particle reads its stencil from LDS, two lanes
// per particle (one half of the axis-0 sum each, combined with a lane
// shuffle) when the piece holds at most 32 particles.
template <int N, typename CT, int C, typename G>
__device__ __forceinline__ void hess_piece(const HessArgs& a, uint32_t cur, uint32_t start, uint32_t count,
                                           u32x4* lds, bool fill) {
    using AT = typename Acc<CT>::type;
    const CT* tile = reinterpret_cast<const CT*>(lds);
    const int tid = threadIdx.x;
    if (cur == a.nbf) {
        for (uint32_t j = tid; j < count; j += HESS_TB) hess_nan<AT, C>(a, long(a.perm[start + j]));
        if (tid == 0) atomicAdd(a.nonfinite, (unsigned long long)count);
        return;
    }
    const bool pair = count <= uint32_t(HESS_TB / 2);
    const int stride = pair ? HESS_TB / 2 : HESS_TB;
    const int o0 = int(compact3(cur >> 2)) * 8;
    const int o1 = int(compact3(cur >> 1)) * 8;
    const int o2 = int(compact3(cur)) * 8;
    if (fill) {
        // the block's 16-byte slots, global -> LDS, all requested at once
        block_dma<N, CT, C, G, HESS_TB>(static_cast<const CT*>(a.grid), a.n0, a.n1, a.P1, a.pitch2, o0, o1, o2, lds);
        __builtin_amdgcn_s_waitcnt(0);
        lds_barrier();
    }
    const uint32_t jlane = pair ? uint32_t(tid >> 1) : uint32_t(tid);
    const int half = pair ? (tid & 1) : 0;
    for (uint32_t j0 = 0; j0 < count; j0 += uint32_t(stride)) {
        const uint32_t jj = j0 + jlane;
        const bool active = jj < count;
        const uint32_t slot = start + (active ? jj : 0u);
        const long p = long(a.perm[slot]);
        const double x[3] = {a.pos_sorted[3 * long(slot)], a.pos_sorted[3 * long(slot) + 1],
                             a.pos_sorted[3 * long(slot) + 2]};
        int cell[3];
        AT w[3][N], wd[3][N], wdd[3][N];
        hess_setup<N, AT>(a, x, cell, w, wd, wdd);  // finite by construction of the tile
        const CT* base = tile + ((cell[0] - o0) * G::R1 + (cell[1] - o1)) * G::LROW + (cell[2] - o2) * C;
        auto rows = [base](int ia, int ib) { return base + (ia * G::R1 + ib) * G::LROW; };
        if (pair) {
            const int ia0 = half * (N / 2);
            AT w0s[N / 2], wd0s[N / 2], wdd0s[N / 2];
#pragma unroll
            for (int k = 0; k < N / 2; ++k) {
                w0s[k] = half ? w[0][N / 2 + k] : w[0][k];
                wd0s[k] = half ? wd[0][N / 2 + k] : wd[0][k];
                wdd0s[k] = half ? wdd[0][N / 2 + k] : wdd[0][k];
            }
            HessSums<AT, C> mine, other;
            hess_planes<N, CT, AT, C, N / 2>(w0s, wd0s, wdd0s, w, wd, wdd,
                                             [&](int k, int ib) { return rows(ia0 + k, ib); }, mine);
#pragma unroll
            for (int m = 0; m < 10; ++m)
#pragma unroll
                for (int c = 0; c < C; ++c) other.s[m][c] = __shfl_xor(mine.s[m][c], 1, 64);
            if (active && half == 0) hess_store<AT, C>(a, p, mine, other);
        } else {
            HessSums<AT, C> lo, hi;
            hess_planes<N, CT, AT, C, N / 2>(w[0], wd[0], wdd[0], w, wd, wdd, rows, lo);
            hess_planes<N, CT, AT, C, N / 2>(w[0] + N / 2, wd[0] + N / 2, wdd[0] + N / 2, w, wd, wdd,
                                             [&](int k, int ib) { return rows(N / 2 + k, ib); }, hi);
            if (active) hess_store<AT, C>(a, p, lo, hi);
        }
    }
}

// LDS-tiled variant: persistent one-wave workgroups over the work items (the
// non-empty Morton tiles of 8^3 cells cut into pieces of at most HESS_ROUNDS
// rounds, so that a crowded tile, a dense cluster of particles, is shared by
// several CUs).  As in the tiled gather, the items are split into one range per
// XCD; a workgroup takes the items of its home range (blockIdx % ITEM_RANGES:
// workgroups are dealt to the XCDs in turn) ITEM_TAKE at a time, then those of
// the other ranges, and consecutive items of one tile reuse its block in LDS.
template <int N, typename CT, int C>
__global__ __launch_bounds__(HESS_TB) void k_gather_hess_tiled(HessArgs a) {
    using G = TileGeom<N, CT, C, 8, false>;   // rows packed densely (hess_planes reads them)
    static_assert(sizeof(CT) != 2 || bf16_rows_fit<N, C, 8, G::LROW>(), "BF16 row reads would leave the LDS row");
    __shared__ u32x4 lds[G::SLOTS];
    // wave-uniform values steer every loop that holds a barrier
    const uint32_t W = __builtin_amdgcn_readfirstlane(a.ctl[0]);
    const uint32_t home = uint32_t(blockIdx.x) % ITEM_RANGES;
    uint32_t prev = 0xffffffffu;  // tile whose block the LDS holds
    for (uint32_t r = 0; r < ITEM_RANGES; ++r) {
        const uint32_t x = (home + r) % ITEM_RANGES;
        const uint32_t lo = item_range_begin(W, x);
        const uint32_t hi = item_range_begin(W, x + 1);
        uint32_t i = item_take_finish<HESS_TB>(item_take_issue(a.ctl, x), nullptr);
        while (lo + i < hi) {
            const uint32_t m = min(ITEM_TAKE, hi - lo - i);
            uint32_t next = 0;
            for (uint32_t k = 0; k < m; ++k) {
                const u32x4 it = a.items[lo + i + k];
                const uint32_t cur = __builtin_amdgcn_readfirstlane(it.x);
                const uint32_t start = __builtin_amdgcn_readfirstlane(it.y);
                const uint32_t count = __builtin_amdgcn_readfirstlane(it.z);
                if (k + 1 == m) next = item_take_issue(a.ctl, x);
                hess_piece<N, CT, C, G>(a, cur, start, count, lds, cur != prev);
                if (cur != a.nbf) prev = cur;
                lds_barrier();  // every LDS read done before a later piece refills it
            }
            i = item_take_finish<HESS_TB>(next, nullptr);
        }
    }
}

template <typename CT>
bool hess_tiled_ok(int N, int C) {
    // FP64 three-component order 6 spills registers in the tiled body: direct
    if (sizeof(CT) == 8 && N == 6 && C == 3) return false;
    auto ok = [](auto g) { return decltype(g)::BYTES <= 65536 && decltype(g)::ALIGNED; };
    if (N == 4) return C == 1 ? ok(TileGeom<4, CT, 1, 8, false>{}) : ok(TileGeom<4, CT, 3, 8, false>{});
    return C == 1 ? ok(TileGeom<6, CT, 1, 8, false>{}) : ok(TileGeom<6, CT, 3, 8, false>{});
}

// Persistent launch: as many workgroups as stay resident (the kernel's
// occupancy, asked once per instance) on every CU.
template <int N, typename CT, int C>
void launch_hess_tiled(int num_cus, hipStream_t s, const HessArgs& a) {
    auto k = k_gather_hess_tiled<N, CT, C>;
    static unsigned per_cu = 0;
    static std::once_flag once;
    std::call_once(once, [&] {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k, HESS_TB, 0) != hipSuccess || v < 1) v = 1;
        per_cu = unsigned(v);
    });
    hipLaunchKernelGGL(k, dim3(per_cu * unsigned(std::max(num_cus, 1))), dim3(HESS_TB), 0, s, a);
}

template <typename CT>
void launch_hess_tiled_ct(int N, int C, int num_cus, hipStream_t s, const HessArgs& a) {
    if (N == 4) {
        if (C == 1) launch_hess_tiled<4, CT, 1>(num_cus, s, a);
        else launch_hess_tiled<4, CT, 3>(num_cus, s, a);
    } else {
        if (C == 1) launch_hess_tiled<6, CT, 1>(num_cus, s, a);
        else launch_hess_tiled<6, CT, 3>(num_cus, s, a);
    }
}

template <typename CT>
void launch_hess_ct(int N, int C, unsigned nb, hipStream_t s, const HessArgs& a) {
    if (N == 4) {
        if (C == 1) hipLaunchKernelGGL((k_gather_hess<4, CT, 1>), dim3(nb), dim3(HESS_B), 0, s, a);
        else hipLaunchKernelGGL((k_gather_hess<4, CT, 3>), dim3(nb), dim3(HESS_B), 0, s, a);
    } else {
        if (C == 1) hipLaunchKernelGGL((k_gather_hess<6, CT, 1>), dim3(nb), dim3(HESS_B), 0, s, a);
        else hipLaunchKernelGGL((k_gather_hess<6, CT, 3>), dim3(nb), dim3(HESS_B), 0, s, a);
    }
}

}  // namespace

bsi_status hessian_run(bsi_field* f, const double* pos, int64_t P, void* u, void* grad, void* hess,
                       hipStream_t s) {
    BSI_CHECK(f->basis == BSI_BASIS_BSPLINE && (f->N == 4 || f->N == 6), BSI_E_UNSUPPORTED,
              "second derivatives are implemented for B-spline fields of orders 4 and 6");
    if (P == 0) return BSI_OK;
    // binned by Morton tiles of 8 cells (at least n/256, so that the bucket
    // table has at most 2^24 entries), for locality of the stencil reads
    const int nmax = std::max(f->n[0], std::max(f->n[1], f->n[2]));
    const int tile = std::max(8, (nmax + 255) / 256);
    const BinLayout l = bin_layout(f, long(P), tile);
    const int coef = f->desc.coef;
    const bool tiled = tile == 8 && (coef == BSI_F64   ? hess_tiled_ok<double>(f->N, f->C)
                                     : coef == BSI_F32 ? hess_tiled_ok<float>(f->N, f->C)
                                                       : hess_tiled_ok<uint16_t>(f->N, f->C));
    // work items of the tiled kernel after the binning's arrays: at most one
    // per non-empty tile plus one per `chunk` particles, then the control
    // words and the per-group item sums
    const uint32_t chunk = uint32_t(HESS_TB) * HESS_ROUNDS;
    const size_t nb = bin_bucket_count(f, tile) + 1;
    const size_t o_items = (l.bytes + 15) / 16 * 16;
    const size_t o_ctl = o_items + (nb + size_t(P) / chunk + 1) * 16;
    const size_t o_sums = o_ctl + ITEM_CTL_WORDS * sizeof(uint32_t);
    const size_t bytes = tiled ? o_sums + (nb + SCAN_CHUNK - 1) / SCAN_CHUNK * sizeof(uint32_t) : l.bytes;
    void* ws = nullptr;
    BSI_TRY(get_workspace(f->ctx->eval_ws, s, bytes, &ws));
    char* w = static_cast<char*>(ws);
    uint32_t* perm = reinterpret_cast<uint32_t*>(w + l.perm);
    double* pos_sorted = reinterpret_cast<double*>(w + l.pos);
    BSI_TRY(bin_run(f, pos, long(P), tile, w + l.grp, perm, pos_sorted, reinterpret_cast<uint32_t*>(w + l.hist),
                    reinterpret_cast<uint32_t*>(w + l.offs), s));
    HessArgs a;
    a.grid = f->grid;
    a.pos_sorted = pos_sorted;
    a.perm = perm;
    a.hist = reinterpret_cast<const uint32_t*>(w + l.hist);
    a.offs = reinterpret_cast<const uint32_t*>(w + l.offs);
    a.nbf = uint32_t(bin_bucket_count(f, tile));
    a.P = long(P);
    a.n0 = f->n[0];
    a.n1 = f->n[1];
    a.n2 = f->n[2];
    a.P1 = f->P[1];
    a.pitch2 = f->pitch2;
    a.ih0 = f->inv_h[0];
    a.ih1 = f->inv_h[1];
    a.ih2 = f->inv_h[2];
    a.u = u;
    a.grad = grad;
    a.hess = hess;
    a.nonfinite = f->counters;
    a.items = nullptr;
    a.ctl = nullptr;
    if (tiled) {
        StageTimer tm(f->ctx, "hess_items", s);
        const uint32_t* hist = a.hist;
        const unsigned ng = unsigned((nb + SCAN_CHUNK - 1) / SCAN_CHUNK);
        uint32_t* sums = reinterpret_cast<uint32_t*>(w + o_sums);
        u32x4* items = reinterpret_cast<u32x4*>(w + o_items);
        uint32_t* ctl = reinterpret_cast<uint32_t*>(w + o_ctl);
        hipLaunchKernelGGL(k_item_sums, dim3(ng), dim3(SCAN_BLOCK), 0, s, hist, long(nb), chunk, sums);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_BLOCK), 0, s, sums, int(ng));
        hipLaunchKernelGGL(k_items, dim3(ng), dim3(SCAN_BLOCK), 0, s, hist, a.offs, long(nb), chunk, sums, items,
                           ctl);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, ctl + ITEM_CTL_STRIDE,
                           long(ITEM_CTL_STRIDE * ITEM_RANGES), 0u);
        a.items = items;
        a.ctl = ctl;
    }
    {
        StageTimer tm(f->ctx, "gather_hess", s);
        if (tiled) {
            const int cus = f->ctx->num_cus;
            if (coef == BSI_F64) launch_hess_tiled_ct<double>(f->N, f->C, cus, s, a);
            else if (coef == BSI_F32) launch_hess_tiled_ct<float>(f->N, f->C, cus, s, a);
            else launch_hess_tiled_ct<uint16_t>(f->N, f->C, cus, s, a);
        } else {
            const unsigned nb = unsigned((P + HESS_B - 1) / HESS_B);
            if (coef == BSI_F64) launch_hess_ct<double>(f->N, f->C, nb, s, a);
            else if (coef == BSI_F32) launch_hess_ct<float>(f->N, f->C, nb, s, a);
            else launch_hess_ct<uint16_t>(f->N, f->C, nb, s, a);
        }
    }
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

}  // namespace bsi
