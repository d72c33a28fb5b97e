"""Pins of oracle.methods (Lagrange, linear, Hermite matrices), the oracle's
Lagrange evaluation and its cubic Hermite interpolation (oracle.hermite).

Pins: the Hermite matrix printed in Section 2 (golden file) and the Hermite
conditions of Section 2 (values and derivatives at both cell ends); for
Lagrange the interpolation property at the nodes, an independent polynomial
fit through the same nodes (numpy), reproduction of polynomials of degree
N - 1 and failure at degree N, and C^0 continuity with a jump in the first
derivative (Table 2: n = N - 1, continuity 0 for even N); linear = the order-2
B-spline; the 3D Lagrange and Hermite interpolants reproduce grid values (and
for Hermite grid derivatives) and polynomials of degree N - 1 exactly, and a
Hermite error of one mode matches an independent Hermite spline (scipy).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle.methods import lagrange_matrix, hermite_matrix, lagrange_nodes, to_f64
from oracle.bspline import bspline_matrix, derivative_matrix
from oracle import evaluate, prefilter, hermite
from oracle.symbol import NONE

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hermite_matrix_printed.txt")


def _poly(row, x):
    return sum(c * x ** i for i, c in enumerate(row))


def test_hermite_matrix_is_the_printed_one():
    with open(GOLDEN) as fh:
        lines = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    _, order, _, scale = lines[0]
    printed = [[Fraction(int(v), int(scale)) for v in row] for row in lines[1:1 + int(order)]]
    assert hermite_matrix(4) == printed


@pytest.mark.parametrize("N", [2, 4, 6])
def test_hermite_conditions(N):
    # row r of M is the basis polynomial of data item r: its l-th derivative at
    # point p is 1 for the item (p, l) and 0 for every other item
    from oracle.methods import hermite_data_rows
    M = hermite_matrix(N)
    items = hermite_data_rows(N)
    for r in range(N):
        for q, (point, l) in enumerate(items):
            d = M[r]
            for _ in range(l):
                d = [(i + 1) * d[i + 1] for i in range(len(d) - 1)] or [Fraction(0)]
            assert _poly(d, Fraction(point)) == (1 if q == r else 0)


@pytest.mark.parametrize("N", [2, 4, 6])
def test_lagrange_interpolates_nodes_and_matches_polyfit(N):
    M = lagrange_matrix(N)
    nodes = lagrange_nodes(N)
    for j in range(N):
        for k, x in enumerate(nodes):
            assert _poly(M[j], x) == (1 if j == k else 0)
    # an independent construction: numpy's polynomial fit through the nodes of
    # a random data vector equals b^T M xbar
    rng = np.random.default_rng(N)
    b = rng.normal(size=N)
    fit = np.polynomial.polynomial.polyfit([float(x) for x in nodes], b, N - 1)
    assert np.allclose(b @ to_f64(M), fit, atol=1e-12)


def test_linear_is_the_order_two_bspline():
    assert lagrange_matrix(2) == bspline_matrix(2)


@pytest.mark.parametrize("N", [2, 4, 6])
def test_lagrange_polynomial_reproduction_and_continuity(N):
    M = lagrange_matrix(N)
    nodes = lagrange_nodes(N)
    for deg in range(N + 1):
        # sum_j w_j(t) p(node_j) = p(t) exactly for deg <= N - 1 (Table 2: n = N - 1)
        ts = [Fraction(k, 7) for k in range(7)]
        ok = all(sum(_poly(M[j], t) * nodes[j] ** deg for j in range(N)) == t ** deg for t in ts)
        assert ok == (deg <= N - 1)
    # C^0: a grid point that is stencil point j + 1 of a cell is point j of the
    # next cell, and its weight is continuous there (w_{j+1}(1) = w_j(0)); the
    # first point leaves and the last enters with weight 0; the derivative of
    # the weight jumps (continuity 0 for even N, Table 2)
    M1 = derivative_matrix(M, 1)
    assert all(_poly(M[j + 1], Fraction(1)) == _poly(M[j], Fraction(0)) for j in range(N - 1))
    assert _poly(M[0], Fraction(1)) == 0 and _poly(M[N - 1], Fraction(0)) == 0
    if N > 2:
        assert any(_poly(M1[j + 1], Fraction(1)) != _poly(M1[j], Fraction(0)) for j in range(N - 1))


def _grid_points(n, count, seed):
    rng = np.random.default_rng(seed)
    g = rng.integers(0, n, size=(count, 3))
    return g, g * (2 * np.pi / n)


@pytest.mark.parametrize("N", [2, 4, 6])
def test_lagrange_3d_interpolates_grid_values(N):
    n = 12
    uhat = synth.kolmogorov_spectrum(n, 3, seed=31)
    vals = prefilter(uhat, N, NONE)                      # c = 1: the field's grid values
    assert np.allclose(vals, np.fft.irfftn(uhat, s=(n, n, n), axes=(1, 2, 3), norm="forward"))
    g, pos = _grid_points(n, 200, 32)
    u, _ = evaluate(vals, pos, N, basis="lagrange")
    want = vals[:, g[:, 0], g[:, 1], g[:, 2]].T
    assert np.max(np.abs(u - want)) < 1e-13


@pytest.mark.parametrize("N", [2, 4, 6])
def test_lagrange_3d_polynomial_reproduction(N):
    # a polynomial of degree N - 1 per axis (sampled on the grid, away from
    # the periodic wrap) and its gradient are reproduced to rounding
    n = 24
    L = 2 * np.pi
    h = L / n
    x = np.arange(n) * h
    p = lambda s, d: s ** d
    dg = N - 1
    grid = (p(x, dg)[:, None, None] * p(x, 1)[None, :, None] * np.ones(n)[None, None, :])[None]
    rng = np.random.default_rng(33)
    pos = rng.uniform(N * h, L - N * h, size=(300, 3))
    u, g = evaluate(grid, pos, N, basis="lagrange")
    want = pos[:, 0] ** dg * pos[:, 1]
    assert np.max(np.abs(u[:, 0] - want)) < 1e-9 * np.max(np.abs(want))
    gx = dg * pos[:, 0] ** (dg - 1) * pos[:, 1] if dg > 0 else 0 * pos[:, 0]
    assert np.max(np.abs(g[:, 0, 0] - gx)) < 1e-8 * max(1.0, np.max(np.abs(gx)))
    assert np.max(np.abs(g[:, 0, 1] - pos[:, 0] ** dg)) < 1e-8 * np.max(np.abs(pos[:, 0] ** dg))


def test_hermite_3d_interpolates_values_and_derivatives_at_nodes():
    n = 12
    uhat = synth.kolmogorov_spectrum(n, 3, seed=35)
    dg = hermite.derivative_grids(uhat)
    g, pos = _grid_points(n, 150, 36)
    u, gr = hermite.evaluate_hermite(dg, pos)
    assert np.max(np.abs(u - dg[(0, 0, 0)][:, g[:, 0], g[:, 1], g[:, 2]].T)) < 1e-13
    ih = n / (2 * np.pi)
    for d, a in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        want = dg[a][:, g[:, 0], g[:, 1], g[:, 2]].T * ih
        assert np.max(np.abs(gr[:, :, d] - want)) < 1e-12 * np.max(np.abs(want))
    # the derivative fields are the spectral derivatives: compare with a
    # direct truncated Fourier sum of the gradient at grid points
    from pins import full_fourier_sum
    _, ex = full_fourier_sum(uhat, pos, grad=True)
    assert np.max(np.abs(gr - ex)) < 1e-11 * np.max(np.abs(ex))


def test_hermite_3d_cubic_reproduction():
    # derivative fields of a cubic polynomial in each coordinate: the Hermite
    # interpolant reproduces it exactly (n = N - 1 = 3)
    n = 16
    h = 1.0
    x = np.arange(n, dtype=np.float64)
    f = lambda s: 0.5 * s ** 3 - s ** 2 + 0.25 * s
    df = lambda s: 1.5 * s ** 2 - 2 * s + 0.25
    fx = {0: f(x), 1: df(x)}
    gy = {0: x ** 2, 1: 2 * x}
    dg = {a: (fx[a[0]][:, None, None] * gy[a[1]][None, :, None] * (1.0 if a[2] == 0 else 0.0)
              * np.ones(n)[None, None, :])[None] for a in hermite.ORDERS}
    rng = np.random.default_rng(37)
    L = 2 * np.pi
    pos = rng.uniform(1.0, n - 2.0, size=(200, 3)) * (L / n)
    s = pos * (n / L)
    u, gr = hermite.evaluate_hermite(dg, pos)
    want = f(s[:, 0]) * s[:, 1] ** 2
    assert np.max(np.abs(u[:, 0] - want)) < 1e-10 * np.max(np.abs(want))
    assert np.max(np.abs(gr[:, 0, 0] - df(s[:, 0]) * s[:, 1] ** 2 * (n / L))) < 1e-9 * np.max(np.abs(want))


@pytest.mark.parametrize("kappa", [1 / 8, 1 / 3, 3 / 8])
def test_hermite_mode_error_matches_scipy_hermite_spline(kappa):
    # 1D: interpolate phi = cos(2 pi kappa s) on a periodic grid with the
    # oracle's Hermite matrix and with scipy's CubicHermiteSpline (an
    # independent implementation); the squared L2 errors of the value and the
    # first derivative agree
    from scipy.interpolate import CubicHermiteSpline
    from pins import gauss_legendre_cells
    q = 24
    s = np.arange(q + 1, dtype=np.float64)
    y = np.cos(2 * np.pi * kappa * s)
    dy = -2 * np.pi * kappa * np.sin(2 * np.pi * kappa * s)
    spl = CubicHermiteSpline(s, y, dy)
    xq, wq = gauss_legendre_cells(q, 8)
    cell = np.floor(xq).astype(int)
    t = xq - cell
    M = to_f64(hermite_matrix(4))
    M1 = to_f64(derivative_matrix(hermite_matrix(4), 1))
    pw = np.stack([t ** i for i in range(4)], axis=-1)
    b = np.stack([y[cell], dy[cell], y[cell + 1], dy[cell + 1]], axis=-1)
    ours = np.sum(b * (pw @ M.T), axis=-1)
    ours1 = np.sum(b * (pw @ M1.T), axis=-1)
    assert np.max(np.abs(ours - spl(xq))) < 1e-13
    assert np.max(np.abs(ours1 - spl(xq, 1))) < 1e-12
