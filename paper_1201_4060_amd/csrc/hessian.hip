// Second derivatives of the interpolant, with u and grad u.
//
// Section 2: the l-th derivative of the interpolant on a cell uses the matrix
// M^(l) = M D^l; here l = 2 gives the weights w''_j(t).  In three dimensions
// (Section 3) the mixed derivative d2/dx_i dx_j takes the first-derivative
// weights on axes i and j, and d2/dx_i^2 the second-derivative weights on
// axis i; every factor carries the chain factor n/L of its axis.  The
// particles are binned as for the evaluation (Morton tiles) and then gathered
// one lane per particle straight from the grid, the contraction reducing axis
// 2 first, then axis 1, then axis 0 (the Table 1 idea), with six per-plane
// partial sums per component instead of three.
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
    long P;
    int n0, n1, n2, P1;
    long pitch2;
    double ih0, ih1, ih2;
    void* u;
    void* grad;  // or nullptr
    void* hess;
    unsigned long long* nonfinite;
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
    if (P == 0) return BSI_OK;
    // binned by Morton tiles of 8 cells (at least n/256, so that the bucket
    // table has at most 2^24 entries), for locality of the stencil reads
    const int nmax = std::max(f->n[0], std::max(f->n[1], f->n[2]));
    const int tile = std::max(8, (nmax + 255) / 256);
    const BinLayout l = bin_layout(f, long(P), tile);
    void* ws = nullptr;
    BSI_TRY(get_workspace(f->ctx->eval_ws, s, l.bytes, &ws));
    char* w = static_cast<char*>(ws);
    uint32_t* perm = reinterpret_cast<uint32_t*>(w + l.perm);
    double* pos_sorted = reinterpret_cast<double*>(w + l.pos);
    BSI_TRY(bin_run(f, pos, long(P), tile, w + l.grp, perm, pos_sorted, reinterpret_cast<uint32_t*>(w + l.hist),
                    reinterpret_cast<uint32_t*>(w + l.offs), s));
    HessArgs a;
    a.grid = f->grid;
    a.pos_sorted = pos_sorted;
    a.perm = perm;
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
    const unsigned nb = unsigned((P + HESS_B - 1) / HESS_B);
    {
        StageTimer tm(f->ctx, "gather_hess", s);
        if (f->desc.coef == BSI_F64) launch_hess_ct<double>(f->N, f->C, nb, s, a);
        else if (f->desc.coef == BSI_F32) launch_hess_ct<float>(f->N, f->C, nb, s, a);
        else launch_hess_ct<uint16_t>(f->N, f->C, nb, s, a);
    }
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

}  // namespace bsi
