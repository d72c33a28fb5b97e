"""Evaluation of the B-spline interpolant and its first derivatives.

Test infrastructure only (see package doc).

Grid coordinates.  The paper rescales space so the grid spacing is one
(Section 5).  A position x_d in a box of length L_d with n_d points has grid
coordinate s_d = x_d * (n_d / L_d).  With f = floor(s) and t = s - f, the
stencil of an order-N method (N even) is the N nearest points
x_j = floor(x - N/2 + j), j = 1..N (Section 5), i.e. f - N/2 + 1 + j for
0-based j = 0..N-1, taken modulo n_d on the periodic grid.

Rounding (a reading, the paper is silent): s is one round-to-nearest FP64
product of x and inv_h = n/L (inv_h itself one FP64 division), f = floor(s),
t = s - f in FP64, and the cell is the exact Euclidean remainder of f by n.
numpy performs each of these as a single IEEE operation, without fused
multiply-add.

Weights.  Section 2: the interpolant on a cell is b^T M xbar with
xbar = (1, t, ..., t^(N-1)); the l-th derivative uses M^(l) = M D^l.  In the
Section 5 convolution form the weight of stencil point j is
w_j(t) = sum_i M[j][i] t^i.  Derivatives with respect to x pick up the chain
factor n/L.

Three dimensions.  Section 3: u~ = B x1 (M xbar) x2 (M ybar) x3 (M zbar) and a
first derivative replaces one factor by M^(1).  Here that is written out as the
plain triple sum over the N^3 stencil, sum_{a,b,e} w0[a] w1[b] w2[e] u_B[...],
without the Table 1 reordering (any order is mathematically equal, Section 3).
A vector field is handled per component (Section 3, last paragraph).
"""
import numpy as np

from .bspline import bspline_matrix, derivative_matrix
from .methods import lagrange_matrix, to_f64

BASES = ("bspline", "lagrange")


def basis_matrices(N, basis="bspline", l=1):
    """M and M^(l) = M D^l (Section 2) of the basis, rounded to float64 once.

    bspline  : M_(N) of Section 7 (the coefficient grid from the prefilter)
    lagrange : Lagrange interpolation through the N nearest points (Section 8;
               N = 2 is linear interpolation), on the grid values themselves
    """
    if basis == "bspline":
        M = bspline_matrix(N)
    elif basis == "lagrange":
        M = lagrange_matrix(N)
    else:
        raise ValueError(f"unknown basis {basis!r}")
    return to_f64(M), to_f64(derivative_matrix(M, l))

TWO_PI = 2.0 * 3.141592653589793


def inv_spacing(n, L):
    """inv_h = n / L as one FP64 division."""
    return float(n) / float(L)


def cells(pos, shape, lengths=(TWO_PI, TWO_PI, TWO_PI)):
    """Cell index and offset per particle and axis.

    Returns (cell int64 [P][3], t float64 [P][3], finite bool [P]).  A particle
    has no cell when one of its grid coordinates s is not finite (a non-finite
    position, or a finite one so large that x * n/L overflows); such rows get
    cell 0, t 0 and finite=False.
    """
    pos = np.asarray(pos, dtype=np.float64)
    P = pos.shape[0]
    with np.errstate(over="ignore", invalid="ignore"):
        svals = np.stack([pos[:, d] * inv_spacing(shape[d], lengths[d]) for d in range(3)], axis=1)
    finite = np.isfinite(svals).all(axis=1)
    cell = np.zeros((P, 3), dtype=np.int64)
    t = np.zeros((P, 3), dtype=np.float64)
    for d in range(3):
        s = np.where(finite, svals[:, d], 0.0)
        f = np.floor(s)
        t[:, d] = s - f
        r = np.fmod(f, float(shape[d]))          # exact remainder, sign of f
        r = np.where(r < 0, r + shape[d], r)
        cell[:, d] = r.astype(np.int64)
    return cell, t, finite


def weights(t, N, inv_h=1.0, basis="bspline"):
    """w[P][N] and w'[P][N] for offsets t[P] (Section 2 matrices, Section 5 form)."""
    M, M1 = basis_matrices(N, basis, 1)
    powers = np.stack([t ** i for i in range(N)], axis=-1)     # [P][N]
    w = powers @ M.T
    wd = (powers @ M1.T) * inv_h
    return w, wd


def weights2(t, N, inv_h=1.0, basis="bspline"):
    """Second-derivative weights w''[P][N]: Section 2 with l = 2, M^(2) = M D^2,
    times the chain factor (n/L)^2."""
    _, M2 = basis_matrices(N, basis, 2)
    powers = np.stack([t ** i for i in range(N)], axis=-1)
    return (powers @ M2.T) * (inv_h * inv_h)


def stencil_indices(cell_d, N, n):
    """Periodic grid indices of the N stencil points along one axis, [P][N]."""
    j = np.arange(N, dtype=np.int64)
    return np.mod(cell_d[:, None] - N // 2 + 1 + j[None, :], n)


def evaluate(grid, pos, N, lengths=(TWO_PI, TWO_PI, TWO_PI), derivatives=True, basis="bspline"):
    """Interpolate u and grad u at positions.

    grid : float64 [C][n0][n1][n2] B-spline coefficients (output of prefilter),
           or grid values for basis="lagrange" (prefilter with variant NONE)
    pos  : float64 [P][3]
    Returns u [P][C] and (if derivatives) grad [P][C][3] with
    grad[p][c][d] = d u_c / d x_d.  Particles with a non-finite coordinate get NaN.
    """
    if N % 2:
        raise ValueError("only even spline orders are supported")
    grid = np.asarray(grid, dtype=np.float64)
    C, n0, n1, n2 = grid.shape
    shape = (n0, n1, n2)
    pos = np.asarray(pos, dtype=np.float64)
    P = pos.shape[0]
    cell, t, finite = cells(pos, shape, lengths)
    W, Wd, idx = [], [], []
    for d in range(3):
        w, wd = weights(t[:, d], N, inv_spacing(shape[d], lengths[d]), basis)
        W.append(w)
        Wd.append(wd)
        idx.append(stencil_indices(cell[:, d], N, shape[d]))
    flat = grid.reshape(C, -1)
    u = np.zeros((P, C), dtype=np.float64)
    grad = np.zeros((P, C, 3), dtype=np.float64) if derivatives else None
    for a in range(N):
        for b in range(N):
            for e in range(N):
                lin = (idx[0][:, a] * n1 + idx[1][:, b]) * n2 + idx[2][:, e]
                vals = flat[:, lin].T                          # [P][C]
                u += (W[0][:, a] * W[1][:, b] * W[2][:, e])[:, None] * vals
                if derivatives:
                    grad[:, :, 0] += (Wd[0][:, a] * W[1][:, b] * W[2][:, e])[:, None] * vals
                    grad[:, :, 1] += (W[0][:, a] * Wd[1][:, b] * W[2][:, e])[:, None] * vals
                    grad[:, :, 2] += (W[0][:, a] * W[1][:, b] * Wd[2][:, e])[:, None] * vals
    if not finite.all():
        u[~finite] = np.nan
        if derivatives:
            grad[~finite] = np.nan
    return (u, grad) if derivatives else u


# the six distinct second derivatives d2/dx_i dx_j, i <= j, in this order
HESS_PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def evaluate_hessian(grid, pos, N, lengths=(TWO_PI, TWO_PI, TWO_PI)):
    """u, grad u and the second derivatives of the interpolant at positions.

    Section 2: the l-th derivative of the interpolant on a cell uses M^(l) = M D^l;
    in three dimensions (Section 3) a mixed second derivative d2/dx_i dx_j
    replaces the weights of axes i and j by their first-derivative weights, and
    d2/dx_i^2 those of axis i by its second-derivative weights.  Plain triple sum
    over the N^3 stencil, as in evaluate().

    Returns u [P][C], grad [P][C][3] and hess [P][C][6] with hess[p][c][m] =
    d2 u_c / dx_i dx_j for (i, j) = HESS_PAIRS[m].  Particles with a non-finite
    coordinate get NaN.
    """
    if N % 2:
        raise ValueError("only even spline orders are supported")
    grid = np.asarray(grid, dtype=np.float64)
    C, n0, n1, n2 = grid.shape
    shape = (n0, n1, n2)
    pos = np.asarray(pos, dtype=np.float64)
    P = pos.shape[0]
    cell, t, finite = cells(pos, shape, lengths)
    W, Wd, Wdd, idx = [], [], [], []
    for d in range(3):
        ih = inv_spacing(shape[d], lengths[d])
        w, wd = weights(t[:, d], N, ih)
        W.append(w)
        Wd.append(wd)
        Wdd.append(weights2(t[:, d], N, ih))
        idx.append(stencil_indices(cell[:, d], N, shape[d]))
    flat = grid.reshape(C, -1)
    u = np.zeros((P, C))
    grad = np.zeros((P, C, 3))
    hess = np.zeros((P, C, 6))
    for a in range(N):
        for b in range(N):
            for e in range(N):
                lin = (idx[0][:, a] * n1 + idx[1][:, b]) * n2 + idx[2][:, e]
                vals = flat[:, lin].T
                j = (a, b, e)
                u += (W[0][:, a] * W[1][:, b] * W[2][:, e])[:, None] * vals
                for d in range(3):
                    f = [W[k][:, j[k]] for k in range(3)]
                    f[d] = Wd[d][:, j[d]]
                    grad[:, :, d] += (f[0] * f[1] * f[2])[:, None] * vals
                for m, (p_, q_) in enumerate(HESS_PAIRS):
                    f = [W[k][:, j[k]] for k in range(3)]
                    if p_ == q_:
                        f[p_] = Wdd[p_][:, j[p_]]
                    else:
                        f[p_] = Wd[p_][:, j[p_]]
                        f[q_] = Wd[q_][:, j[q_]]
                    hess[:, :, m] += (f[0] * f[1] * f[2])[:, None] * vals
    if not finite.all():
        u[~finite] = np.nan
        grad[~finite] = np.nan
        hess[~finite] = np.nan
    return u, grad, hess
