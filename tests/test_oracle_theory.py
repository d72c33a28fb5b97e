"""Pins of oracle.theory: the per-mode errors of Section 5 (eq. l2-error and
l2-error-der) for the four methods of the comparison (Section 8: B-spline with
both c, Lagrange, Hermite, linear) -- the curves of Figs 3 and 4.

Pins: two independent evaluations of the alias series (closed-form transforms
with a tail term, and the exact sum by Poisson summation) agree; the B-spline
agrees with the series of F[B_(N)] = sinc^N written out; linear interpolation
has textbook closed forms; every curve equals the L2 error of the actual
interpolant of one mode integrated by quadrature, the interpolant built
independently (Cox-de Boor B-splines, numpy polynomial fits, numpy's linear
interpolation, scipy's Hermite spline); the small-kappa slopes are the orders
of Table 2 (n + 1 for the value, one less per derivative); the Hermite error
properties of Section 6; the continuity column of Table 2.
"""
import numpy as np
import pytest

from oracle import theory as T
from oracle.symbol import L2OPT, INTERP
from pins import bspline_float, bspline_deriv_float, bspline_deriv2_float, gauss_legendre_cells

KAPPAS = np.array([0.2, 1 / 3, 0.45])

METHODS = {
    "bspline4-l2opt": lambda: T.bspline_method(4, L2OPT),
    "bspline4-interp": lambda: T.bspline_method(4, INTERP),
    "bspline6-l2opt": lambda: T.bspline_method(6, L2OPT),
    "lagrange4": lambda: T.lagrange_method(4),
    "lagrange6": lambda: T.lagrange_method(6),
    "linear": lambda: T.lagrange_method(2),
    "hermite4": lambda: T.hermite_method(4),
}


@pytest.mark.parametrize("name", sorted(METHODS))
@pytest.mark.parametrize("l", [0, 1, 2])
def test_series_with_tail_equals_poisson_sum(name, l):
    m = METHODS[name]()
    a = T.mode_error(m, KAPPAS, l)
    b = T.mode_error_poisson(m, KAPPAS, l)
    if not np.isfinite(b).all():
        assert not np.isfinite(a).any()
        assert m.continuity() < l - 1
        return
    assert np.max(np.abs(a - b) / b) < 1e-9


@pytest.mark.parametrize("N,variant", [(4, L2OPT), (4, INTERP), (6, L2OPT), (6, INTERP)])
@pytest.mark.parametrize("l", [0, 1, 2])
def test_bspline_equals_sinc_series(N, variant, l):
    m = T.bspline_method(N, variant)
    k = np.array([0.05, 0.2, 1 / 3, 0.45])
    a = T.mode_error(m, k, l)
    b = T.mode_error_1d(k, N, variant, l, terms=20000)
    assert np.max(np.abs(a - b) / b) < 1e-6


def test_linear_closed_forms():
    # hat kernel: F = sinc^2, sum_i sinc^4(kappa + i) = (2 + cos 2 pi kappa)/3,
    # and its derivative (a +-1 step pair) gives 1 - sinc^2 for l = 1
    k = np.linspace(0.02, 0.5, 25)
    s2 = np.sinc(k) ** 2
    m = T.lagrange_method(2)
    e0 = 1 - 2 * s2 + (2 + np.cos(2 * np.pi * k)) / 3
    assert np.max(np.abs(T.mode_error(m, k, 0) - e0) / e0) < 1e-9
    assert np.max(np.abs(T.mode_error(m, k, 1) - (1 - s2)) / (1 - s2)) < 1e-9
    assert np.isinf(T.mode_error(m, k, 2)).all()


def _quadrature_error(values, exact, q):
    x, w = gauss_legendre_cells(q, 16)
    num = np.sum(w * np.abs(values(x) - exact(x)) ** 2)
    return num / np.sum(w * np.abs(exact(x)) ** 2)


def _mode(kappa, l):
    return lambda x: (2j * np.pi * kappa) ** l * np.exp(2j * np.pi * kappa * x)


@pytest.mark.parametrize("p,q", [(1, 8), (1, 3), (3, 8), (5, 12)])
@pytest.mark.parametrize("N,variant", [(4, L2OPT), (4, INTERP), (6, L2OPT)])
def test_bspline_curve_is_the_interpolants_error(p, q, N, variant):
    # periodic grid of q points; the prefilter of one DFT mode multiplies it by
    # c(kappa) (Section 7), so the interpolant is c sum_j phi(j) B(x - j)
    kappa = p / q
    c = T.c_value(kappa, N, variant)[0]
    j = np.arange(-2 * N, q + 2 * N)
    coef = c * np.exp(2j * np.pi * kappa * j)
    fns = (bspline_float, bspline_deriv_float, bspline_deriv2_float)
    for l in (0, 1, 2):
        f = fns[l]
        got = _quadrature_error(lambda x: (coef[None, :] * f(N, x[:, None] - j[None, :])).sum(axis=1),
                                _mode(kappa, l), q)
        want = T.mode_error(T.bspline_method(N, variant), kappa, l)[0]
        assert abs(got - want) < 1e-9 * want


def _piecewise_fit(kappa, N, q, l):
    # Lagrange: on cell [g, g+1) the polynomial through the N nearest points
    # g - N/2 + 1 .. g + N/2 (Section 5), fitted by numpy, differentiated l times
    P = np.polynomial.polynomial
    nodes = np.arange(N) - N // 2 + 1
    phi = lambda s: np.exp(2j * np.pi * kappa * s)
    def values(x):
        out = np.empty(x.shape, dtype=np.complex128)
        cell = np.floor(x).astype(int)
        for g in np.unique(cell):
            m = cell == g
            s = g + nodes
            cr = P.polyfit(nodes, phi(s).real, N - 1)
            ci = P.polyfit(nodes, phi(s).imag, N - 1)
            t = x[m] - g
            out[m] = P.polyval(t, P.polyder(cr, l)) + 1j * P.polyval(t, P.polyder(ci, l))
        return out
    return values


@pytest.mark.parametrize("p,q", [(1, 8), (1, 3), (3, 8)])
@pytest.mark.parametrize("N", [2, 4, 6])
def test_lagrange_curve_is_the_interpolants_error(p, q, N):
    kappa = p / q
    for l in (0, 1):
        got = _quadrature_error(_piecewise_fit(kappa, N, q, l), _mode(kappa, l), q)
        want = T.mode_error(T.lagrange_method(N), kappa, l)[0]
        assert abs(got - want) < 1e-9 * want
    if N == 2:   # and the plain linear interpolation of numpy
        xs = np.arange(q + 1)
        y = np.exp(2j * np.pi * kappa * xs)
        lin = lambda x: np.interp(x, xs, y.real) + 1j * np.interp(x, xs, y.imag)
        got = _quadrature_error(lin, _mode(kappa, 0), q)
        assert abs(got - T.mode_error(T.lagrange_method(2), kappa, 0)[0]) < 1e-9 * got


@pytest.mark.parametrize("p,q", [(1, 8), (1, 3), (3, 8), (5, 12)])
def test_hermite_curve_is_the_interpolants_error(p, q):
    from scipy.interpolate import CubicHermiteSpline
    kappa = p / q
    xs = np.arange(q + 1, dtype=np.float64)
    y = np.exp(2j * np.pi * kappa * xs)
    dy = 2j * np.pi * kappa * y
    sr = CubicHermiteSpline(xs, y.real, dy.real)
    si = CubicHermiteSpline(xs, y.imag, dy.imag)
    for l in (0, 1, 2):
        got = _quadrature_error(lambda x: sr(x, l) + 1j * si(x, l), _mode(kappa, l), q)
        want = T.mode_error(T.hermite_method(4), kappa, l)[0]
        assert abs(got - want) < 1e-9 * want


@pytest.mark.parametrize("name,n", [("bspline4-l2opt", 3), ("bspline6-l2opt", 5), ("lagrange4", 3),
                                    ("lagrange6", 5), ("linear", 1), ("hermite4", 3)])
def test_small_kappa_slopes_are_table2_orders(name, n):
    # squared error ~ kappa^(2 (n + 1 - l)): order of convergence n + 1 (Section 8)
    m = METHODS[name]()
    for l in (0, 1):
        e1, e2 = (T.mode_error(m, np.array([k]), l)[0] for k in (0.005, 0.01))
        slope = np.log(e2 / e1) / np.log(2.0)
        assert abs(slope - 2 * (n + 1 - l)) < 0.05, (name, l, slope)


def test_continuity_column_of_table2():
    assert T.bspline_method(4).continuity() == 2 and T.bspline_method(6).continuity() == 4
    assert T.lagrange_method(4).continuity() == 0 and T.lagrange_method(6).continuity() == 0
    assert T.lagrange_method(2).continuity() == 0
    assert T.hermite_method(4).continuity() == 1          # (N - 2)/2


@pytest.mark.parametrize("kappa", [1 / 8, 1 / 3, 3 / 8])
def test_hermite_error_properties(kappa):
    # Section 6: on every cell the first-derivative error has no constant
    # component, and for N = 4 the second-derivative error has neither a
    # constant nor a linear one
    from scipy.interpolate import CubicHermiteSpline
    q = 8
    xs = np.arange(q + 1, dtype=np.float64)
    y = np.cos(2 * np.pi * kappa * xs)
    s = CubicHermiteSpline(xs, y, -2 * np.pi * kappa * np.sin(2 * np.pi * kappa * xs))
    x, w = np.polynomial.legendre.leggauss(12)
    t = 0.5 * (x + 1)
    w = 0.5 * w
    for g in range(q):
        e1 = s(g + t, 1) + 2 * np.pi * kappa * np.sin(2 * np.pi * kappa * (g + t))
        e2 = s(g + t, 2) + (2 * np.pi * kappa) ** 2 * np.cos(2 * np.pi * kappa * (g + t))
        assert abs(np.sum(w * e1)) < 1e-13
        assert abs(np.sum(w * e2)) < 1e-12 and abs(np.sum(w * t * e2)) < 1e-12


def test_values_at_one_third():
    # values derived from eq. l2-error / l2-error-der for the B-spline at the
    # dealiasing cut-off kappa = 1/3 (Section 8); 4 significant digits
    want = {(4, L2OPT, 0): 3.909e-3, (4, INTERP, 0): 7.596e-3, (6, L2OPT, 0): 2.441e-4,
            (6, INTERP, 0): 4.830e-4, (4, L2OPT, 1): 1.584e-2, (4, INTERP, 1): 1.812e-2,
            (6, L2OPT, 1): 9.772e-4, (6, INTERP, 1): 1.194e-3}
    for (N, v, l), w in want.items():
        got = T.mode_error(T.bspline_method(N, v), np.array([1 / 3]), l)[0]
        assert abs(got - w) < 6e-4 * w, (N, v, l, got)


def test_comparison_ordering_and_curves():
    # Figs 3-4: at the cut-off the B-spline (L2-optimal c) is close to Hermite
    # and well below Lagrange and linear; the L2-optimal c beats the
    # interpolating one at every kappa (optimality, Section 7)
    k = np.linspace(0.01, 0.5, 50)
    cur = T.figure_curves(k)
    i3 = np.argmin(np.abs(k - 1 / 3))
    v = {name: c[0][i3] for name, c in cur.items()}
    assert v["hermite4"] < v["bspline4-l2opt"] < v["bspline4-interp"] < v["lagrange4"] < v["linear"]
    assert np.all(cur["bspline4-l2opt"][0] <= cur["bspline4-interp"][0] * (1 + 1e-12))
    assert np.isinf(cur["lagrange4"][2]).all()          # C^0: the second derivative holds deltas
    assert np.isfinite(cur["hermite4"][2]).all() and np.isfinite(cur["bspline4-l2opt"][2]).all()


def test_3d_product_form_matches_quadrature_for_lagrange():
    # the 3D product form (Section 5) against the oracle's 3D Lagrange
    # evaluation of one mode, integrated by quadrature
    import synth  # noqa: F401
    from oracle import evaluate, prefilter
    from oracle.symbol import NONE
    from pins import full_fourier_sum
    n = 8
    k = (1, -2, 3)
    uhat = np.zeros((1, n, n, n // 2 + 1), dtype=np.complex128)
    uhat[0, k[0] % n, k[1] % n, k[2]] = 0.5
    vals = prefilter(uhat, 4, NONE)
    x, w = gauss_legendre_cells(n, 8)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), axis=-1).reshape(-1, 3) * (2 * np.pi / n)
    W = np.einsum("a,b,c->abc", w, w, w).ravel()
    W /= W.sum()
    u, g = evaluate(vals, X, 4, basis="lagrange")
    ex, gx = full_fourier_sum(uhat, X, grad=True)
    kap = [np.array([kk / n]) for kk in k]
    m = T.lagrange_method(4)
    rel = np.sum(W * (u[:, 0] - ex[:, 0]) ** 2) / np.sum(W * ex[:, 0] ** 2)
    assert abs(rel - T.mode_error_3d(kap, 4, method=m)[0]) < 1e-6 * rel
    for d in range(3):
        rd = np.sum(W * (g[:, 0, d] - gx[:, 0, d]) ** 2) / np.sum(W * gx[:, 0, d] ** 2)
        assert abs(rd - T.mode_error_3d(kap, 4, method=m, deriv_axis=d)[0]) < 1e-6 * rd
