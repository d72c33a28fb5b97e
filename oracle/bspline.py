"""Exact B-spline interpolation matrices.  Test infrastructure only (see package doc).

Conventions (Section 2, the framework u~ = b^T M xbar): row index = stencil
point (which grid value b_j the row weights), column index = power of the
local coordinate t in [0, 1).  Weight of stencil point j at offset t is
w_j(t) = sum_i M[j][i] t^i  (0-based here).
"""
from fractions import Fraction
from math import comb, factorial

import numpy as np


def bspline_matrix(N):
    """M_(N) from the general formula of Section 7, in exact rationals.

    The paper gives, for 1-based row r and column c,
        M_(N),r,c = 1/(N-1)! * Q_{N-1}^{N-c} * sum_{s=r}^{N} (-1)^(s-r) Q_N^{s-r} (N-s)^(N-c)
    with Q the binomial coefficient.  Reading: the term (N-s)^(N-c) at s = N,
    c = N is 0^0 and is taken as 1 (this is what reproduces the last column of
    the printed M_(2), M_(3), M_(4)).  Python's integer 0**0 is 1.
    The surrounding text indexes M_(N),i,j with i the power in one place; the
    printed matrices and this formula both have the row as stencil point,
    which is the reading used here.
    """
    if N < 1:
        raise ValueError("N >= 1")
    M = [[Fraction(0)] * N for _ in range(N)]
    for r in range(1, N + 1):
        for c in range(1, N + 1):
            acc = 0
            for s in range(r, N + 1):
                acc += (-1) ** (s - r) * comb(N, s - r) * (N - s) ** (N - c)
            M[r - 1][c - 1] = Fraction(comb(N - 1, N - c) * acc, factorial(N - 1))
    return M


def derivative_matrix(M, l=1):
    """M^(l) = M D^l (Section 2), exact.

    D maps the coefficient of t^(i+1) onto t^i with factor (i+1): (M D)[j][i] =
    (i+1) M[j][i+1], and the last column is zero.  Applied l times.
    """
    N = len(M)
    out = [row[:] for row in M]
    for _ in range(l):
        nxt = [[Fraction(0)] * N for _ in range(N)]
        for j in range(N):
            for i in range(N - 1):
                nxt[j][i] = (i + 1) * out[j][i + 1]
        out = nxt
    return out


def matrix_f64(N):
    """M_(N) rounded to float64 (each exact rational rounded once)."""
    return np.array([[float(v) for v in row] for row in bspline_matrix(N)],
                    dtype=np.float64)


def derivative_matrix_f64(N, l=1):
    """M_(N)^(l) rounded to float64."""
    return np.array([[float(v) for v in row]
                     for row in derivative_matrix(bspline_matrix(N), l)],
                    dtype=np.float64)
