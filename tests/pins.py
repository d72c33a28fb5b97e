"""Independent mathematical references used to pin the oracle.

Nothing here is imported from ``oracle/``: these are textbook identities for
the centred cardinal B-spline of order N (support [-N/2, N/2], degree N-1),
the N-fold convolution of the unit box B_(1) (Section 7 of the paper):

* truncated-power form (de Boor, "A Practical Guide to Splines"):
      B_N(y) = 1/(N-1)! sum_{k=0}^{N} (-1)^k C(N,k) (y + N/2 - k)_+^(N-1)
* Cox-de Boor recursion for cardinal splines:
      B_N(y) = [(y + N/2) B_{N-1}(y + 1/2) + (N/2 - y) B_{N-1}(y - 1/2)] / (N - 1)
* derivative: B_N'(y) = B_{N-1}(y + 1/2) - B_{N-1}(y - 1/2)
"""
from fractions import Fraction
from math import comb, factorial

import numpy as np


def bspline_exact(N, y):
    """B_N(y) in exact rationals (truncated powers); B_1 is 1 on [-1/2, 1/2)."""
    y = Fraction(y)
    half = Fraction(N, 2)
    acc = Fraction(0)
    for k in range(N + 1):
        z = y + half - k
        if N == 1:
            term = Fraction(1) if z >= 0 else Fraction(0)
        else:
            term = z ** (N - 1) if z > 0 else Fraction(0)
        acc += (-1) ** k * comb(N, k) * term
    return acc / factorial(N - 1)


def bspline_deriv_exact(N, y, order=1):
    """order-th derivative of B_N at y (exact), by the difference identity."""
    y = Fraction(y)
    if order == 0:
        return bspline_exact(N, y)
    h = Fraction(1, 2)
    return (bspline_deriv_exact(N - 1, y + h, order - 1)
            - bspline_deriv_exact(N - 1, y - h, order - 1))


def bspline_float(N, y):
    """B_N(y) for float arrays via the Cox-de Boor recursion (stable, nonnegative)."""
    y = np.asarray(y, dtype=np.float64)
    if N == 1:
        return ((y >= -0.5) & (y < 0.5)).astype(np.float64)
    h = N / 2.0
    return ((y + h) * bspline_float(N - 1, y + 0.5)
            + (h - y) * bspline_float(N - 1, y - 0.5)) / (N - 1)


def bspline_deriv_float(N, y):
    y = np.asarray(y, dtype=np.float64)
    return bspline_float(N - 1, y + 0.5) - bspline_float(N - 1, y - 0.5)


def bspline_deriv2_float(N, y):
    """B_N''(y) from two differences of the Cox-de Boor B_(N-2)."""
    y = np.asarray(y, dtype=np.float64)
    return bspline_float(N - 2, y + 1.0) - 2.0 * bspline_float(N - 2, y) + bspline_float(N - 2, y - 1.0)


def gauss_legendre_cells(n, per_cell):
    """Nodes and weights of a composite Gauss-Legendre rule on [0, n)."""
    x, w = np.polynomial.legendre.leggauss(per_cell)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    nodes = (np.arange(n)[:, None] + x[None, :]).ravel()
    wts = np.tile(w, n)
    return nodes, wts


def full_fourier_sum(uhat, pos, lengths=(2 * np.pi,) * 3, grad=False):
    """Direct truncated Fourier summation u(x) = sum_k uhat_k exp(i k.x).

    uhat is the real-FFT half spectrum [C][n0][n1][n2/2+1]; the sum runs over
    its non-zero entries and their Hermitian partners (k2 > 0 counted twice
    as 2 Re(...); k2 = 0 and k2 = n2/2 entries once each, which is exact when
    the input is Hermitian in those planes).
    """
    C, n0, n1, h = uhat.shape
    n2 = 2 * (h - 1)
    nz = np.nonzero(np.abs(uhat).sum(axis=0))
    k0 = np.where(nz[0] <= n0 // 2, nz[0], nz[0] - n0).astype(np.float64)
    k1 = np.where(nz[1] <= n1 // 2, nz[1], nz[1] - n1).astype(np.float64)
    k2 = nz[2].astype(np.float64)
    wgt = np.where((nz[2] == 0) | (nz[2] == n2 // 2), 1.0, 2.0)
    coef = uhat[:, nz[0], nz[1], nz[2]]                     # [C][K]
    sc = [2 * np.pi / L for L in lengths]
    P = pos.shape[0]
    u = np.zeros((P, C))
    g = np.zeros((P, C, 3)) if grad else None
    step = 2048
    for s in range(0, P, step):
        x = pos[s:s + step]
        ph = (x[:, 0:1] * (k0 * sc[0]) + x[:, 1:2] * (k1 * sc[1])
              + x[:, 2:3] * (k2 * sc[2]))
        e = np.exp(1j * ph) * wgt                            # [p][K]
        val = e @ coef.T                                     # [p][C]
        u[s:s + step] = val.real
        if grad:
            for d, kd in enumerate((k0, k1, k2)):
                g[s:s + step, :, d] = ((1j * kd * sc[d] * e) @ coef.T).real
    return (u, g) if grad else u
