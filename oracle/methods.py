"""Interpolation matrices of the methods the paper compares.  Test infrastructure only.

Section 2 writes every method as u~ = b^T M xbar on a cell, t in [0, 1), with
b = f[u] the method's data and xbar = (1, t, ..., t^(N-1)); the same row =
data item, column = power convention as ``bspline.py``.

* Lagrange interpolation (Section 8, first method): the polynomial of degree
  N-1 through the values at the N nearest grid points, i.e. the stencil of
  Section 5, x_j = floor(x - N/2 + j), j = 1..N, which in the cell's local
  coordinate are the nodes 1 - N/2, ..., N/2.  Row j of M holds the monomial
  coefficients of the j-th Lagrange basis polynomial through those nodes.
  Linear interpolation is the case N = 2.
* Hermite interpolation (Section 2): f = (u(0), u'(0), ..., u^(N/2-1)(0),
  u(1), ..., u^(N/2-1)(1)), and u~ must reproduce those values and
  derivatives at both cell ends (the conditions of Section 2).  With V the
  matrix that maps monomial coefficients a to f[t -> a^T xbar], the condition
  f[u~] = b for every b gives V M^T = I, so M = (V^-1)^T, solved here in exact
  rationals.  The paper prints M for N = 4.
"""
from fractions import Fraction
from math import factorial

import numpy as np


def _poly_mul(p, q):
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def lagrange_nodes(N):
    """Local coordinates of the N stencil points of a cell (Section 5 rule)."""
    return [Fraction(j - N // 2 + 1) for j in range(N)]


def lagrange_matrix(N):
    """M of Lagrange interpolation through the N nearest points, exact (N even)."""
    if N < 2 or N % 2:
        raise ValueError("even N >= 2")
    nodes = lagrange_nodes(N)
    M = []
    for j in range(N):
        poly = [Fraction(1)]
        den = Fraction(1)
        for k in range(N):
            if k != j:
                poly = _poly_mul(poly, [-nodes[k], Fraction(1)])
                den *= nodes[j] - nodes[k]
        M.append([c / den for c in poly])
    return M


def _solve_exact(A):
    """Inverse of a square matrix of Fractions by Gauss-Jordan elimination."""
    n = len(A)
    aug = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        p = aug[col][col]
        aug[col] = [v / p for v in aug[col]]
        for r in range(n):
            if r != col and aug[r][col] != 0:
                f = aug[r][col]
                aug[r] = [a - f * b for a, b in zip(aug[r], aug[col])]
    return [row[n:] for row in aug]


def hermite_data_rows(N):
    """(point, derivative order) of each entry of f, in the Section 2 order."""
    h = N // 2
    return [(0, l) for l in range(h)] + [(1, l) for l in range(h)]


def hermite_matrix(N=4):
    """M of Hermite interpolation with derivatives up to N/2 - 1 at both ends, exact."""
    if N < 2 or N % 2:
        raise ValueError("even N >= 2")
    V = []
    for point, l in hermite_data_rows(N):
        row = []
        for i in range(N):
            # d^l/dt^l t^i at t = point
            if i < l:
                row.append(Fraction(0))
            else:
                row.append(Fraction(factorial(i), factorial(i - l)) * Fraction(point) ** (i - l))
        V.append(row)
    Vinv = _solve_exact(V)
    return [[Vinv[i][j] for i in range(N)] for j in range(N)]    # transpose


def to_f64(M):
    return np.array([[float(v) for v in row] for row in M], dtype=np.float64)
