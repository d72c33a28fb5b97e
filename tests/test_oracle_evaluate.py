"""Pins of oracle.evaluate (stencil, weights, triple sum) and of the whole oracle.

Pins:
* all-lattice brute force on tiny periodic grids: sum over every grid point and
  periodic image of u_B[j] * prod_d B(s_d - j_d), with B from the Cox-de Boor
  recursion (no matrix M, no stencil rule, no floor/fmod cell logic);
* exact reproduction of polynomials of degree <= N-1 (Table 2: n = N-1), with
  coefficients built from the Strang-Fix moments of the B-spline;
* cell/offset edge cases and non-finite positions;
* the per-mode relative L2 error closed form of Section 5 (value and first
  derivatives) for a single 3D mode, measured by Gauss quadrature;
* the orthogonality corollary of Section 5 for a multi-mode Kolmogorov field;
* the convergence order N for u and N-1 for grad u (Section 8).
"""
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import synth
from oracle import evaluate, cells, prefilter, theory, INTERP, L2OPT, TWO_PI
from pins import bspline_float, bspline_deriv_float, gauss_legendre_cells, full_fourier_sum


def _brute_force(grid, pos, N, L=TWO_PI):
    C, n0, n1, n2 = grid.shape
    shape = (n0, n1, n2)
    W, Wd = [], []
    for d in range(3):
        n = shape[d]
        s = pos[:, d] * (n / L)
        g = np.arange(n)
        w = np.zeros((pos.shape[0], n))
        wd = np.zeros((pos.shape[0], n))
        for m in range(-8, 9):                      # periodic images
            y = s[:, None] - (g[None, :] + m * n)
            w += bspline_float(N, y)
            wd += bspline_deriv_float(N, y) * (n / L)
        W.append(w)
        Wd.append(wd)
    u = np.einsum("pa,pb,pe,cabe->pc", W[0], W[1], W[2], grid)
    grad = np.stack([
        np.einsum("pa,pb,pe,cabe->pc", Wd[0], W[1], W[2], grid),
        np.einsum("pa,pb,pe,cabe->pc", W[0], Wd[1], W[2], grid),
        np.einsum("pa,pb,pe,cabe->pc", W[0], W[1], Wd[2], grid)], axis=-1)
    return u, grad


def _edge_positions(rng, n_random):
    L = TWO_PI
    special = np.array([
        [0.0, 0.0, 0.0],
        [L, L, L],
        [np.nextafter(L, 0), np.nextafter(0.0, 1.0), -0.0],
        [-1e-300, -L, 2 * L],
        [-3.7, 13.1, -8.2],
        [L / 8 * 3, L / 10 * 7, L / 12 * 5],          # grid nodes (up to rounding)
    ])
    rnd = rng.uniform(-L, 2 * L, size=(n_random, 3))
    return np.concatenate([special, rnd])


@pytest.mark.parametrize("N", [4, 6])
@pytest.mark.parametrize("shape", [(8, 10, 12), (12, 12, 12)])
def test_all_lattice_brute_force(N, shape):
    rng = np.random.default_rng(5)
    grid = rng.standard_normal((2,) + shape)
    pos = _edge_positions(rng, 40)
    u, g = evaluate(grid, pos, N)
    ub, gb = _brute_force(grid, pos, N)
    scale = np.max(np.abs(grid))
    assert np.max(np.abs(u - ub)) < 1e-12 * scale
    assert np.max(np.abs(g - gb)) < 1e-11 * scale


def _moments(N):
    return {0: Fraction(1), 1: Fraction(0), 2: Fraction(N, 12), 3: Fraction(0),
            4: Fraction(N, 80) + Fraction(N * (N - 1), 48), 5: Fraction(0)}


def _reproducing_coeffs(k, N):
    """q with sum_j w_j(t) q(f + j_rel) = s^k: solve the triangular moment system.

    A monomial J^m of the global index maps to sum_r C(m,r) mu_r s^(m-r).
    """
    mu = _moments(N)
    q = [Fraction(0)] * (k + 1)
    target = [Fraction(0)] * (k + 1)
    target[k] = Fraction(1)
    for m in range(k, -1, -1):          # eliminate from the top degree down
        a = target[m]
        q[m] = a
        for r in range(1, m + 1):
            target[m - r] -= a * comb(m, r) * mu.get(r, Fraction(0))
    return [float(v) for v in q]


@pytest.mark.parametrize("N", [4, 6])
def test_polynomial_reproduction(N):
    n = 32
    degs = (N - 1, 1, N - 2)
    qs = [_reproducing_coeffs(k, N) for k in degs]
    J = np.arange(n, dtype=np.float64)
    vals = [sum(c * J ** m for m, c in enumerate(q)) for q in qs]
    grid = np.einsum("a,b,e->abe", vals[0], vals[1], vals[2])[None]
    rng = np.random.default_rng(9)
    h = TWO_PI / n
    pos = rng.uniform(N * h, (n - N) * h, size=(200, 3))    # away from the wrap
    u, g = evaluate(grid, pos, N)
    s = pos / h
    exact = s[:, 0] ** degs[0] * s[:, 1] ** degs[1] * s[:, 2] ** degs[2]
    dexact = np.stack([
        degs[0] * s[:, 0] ** (degs[0] - 1) * s[:, 1] ** degs[1] * s[:, 2] ** degs[2],
        s[:, 0] ** degs[0] * degs[1] * s[:, 1] ** (degs[1] - 1) * s[:, 2] ** degs[2],
        s[:, 0] ** degs[0] * s[:, 1] ** degs[1] * degs[2] * s[:, 2] ** (degs[2] - 1),
    ], axis=-1) / h
    assert np.max(np.abs(u[:, 0] - exact) / np.abs(exact).max()) < 1e-12
    assert np.max(np.abs(g[:, 0] - dexact) / np.abs(dexact).max()) < 1e-12
    # one degree higher is not reproduced (failure order N)
    q = _reproducing_coeffs(N, N)
    grid2 = np.broadcast_to(sum(c * J ** m for m, c in enumerate(q))[None, None, None, :],
                            (1, n, n, n)).copy()
    u2 = evaluate(grid2, pos, N, derivatives=False)
    assert np.ptp(u2[:, 0] - s[:, 2] ** N) > 1e-6


def test_cells_edges():
    n = 16
    L = TWO_PI
    pos = np.array([[L, 0.0, -0.0],
                    [np.nextafter(0.0, -1.0), np.nextafter(L, 0.0), 3 * L],
                    [-L, 1e300, -1e300]])
    cell, t, fin = cells(pos, (n, n, n))
    assert fin.all()
    assert list(cell[0]) == [0, 0, 0] and list(t[0]) == [0.0, 0.0, 0.0]
    assert cell[1][0] == n - 1 and 0.0 < t[1][0] <= 1.0
    assert cell[1][1] == n - 1
    assert cell[1][2] == 0 and t[1][2] == 0.0
    # huge coordinates: s is an integer-valued double, remainder is exact
    s = 1e300 * (n / L)
    assert cell[2][1] == int(np.fmod(s, n)) and t[2][1] == 0.0
    assert 0 <= cell[2][2] < n


def test_nonfinite_positions_give_nan():
    grid = np.ones((3, 8, 8, 8))
    pos = np.array([[0.1, 0.2, 0.3], [np.nan, 0, 0], [0, np.inf, 0], [1.0, 1.0, -np.inf]])
    u, g = evaluate(grid, pos, 4)
    assert np.allclose(u[0], 1.0) and np.allclose(g[0], 0.0, atol=1e-13)
    assert np.isnan(u[1:]).all() and np.isnan(g[1:]).all()


def _quadrature(n, per_cell):
    x, w = gauss_legendre_cells(n, per_cell)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), axis=-1).reshape(-1, 3)
    Wt = np.einsum("a,b,c->abc", w, w, w).ravel()
    return X * (TWO_PI / n), Wt / Wt.sum()


@pytest.mark.parametrize("N,variant", [(4, L2OPT), (4, INTERP), (6, L2OPT)])
def test_single_mode_error_matches_closed_form(N, variant):
    n = 8
    k = (1, -2, 3)
    uhat = np.zeros((1, n, n, n // 2 + 1), dtype=np.complex128)
    uhat[0, k[0] % n, k[1] % n, k[2]] = 0.5                 # u = cos(k.x)
    grid = prefilter(uhat, N, variant)
    pos, wq = _quadrature(n, 8)
    u, g = evaluate(grid, pos, N)
    ex, gx = full_fourier_sum(uhat, pos, grad=True)
    kap = [np.array([kk / n]) for kk in k]
    rel = np.sum(wq * (u[:, 0] - ex[:, 0]) ** 2) / np.sum(wq * ex[:, 0] ** 2)
    want = theory.mode_error_3d(kap, N, variant)[0]
    assert abs(rel - want) < 1e-6 * want
    for d in range(3):
        rel_d = np.sum(wq * (g[:, 0, d] - gx[:, 0, d]) ** 2) / np.sum(wq * gx[:, 0, d] ** 2)
        want_d = theory.mode_error_3d(kap, N, variant, deriv_axis=d)[0]
        assert abs(rel_d - want_d) < 1e-6 * want_d


@pytest.mark.parametrize("N", [4, 6])
def test_multimode_error_is_spectrum_weighted_sum(N):
    # orthogonality corollary (Section 5) on a Kolmogorov field
    n = 8
    uhat = synth.kolmogorov_spectrum(n, 1, seed=21)
    grid = prefilter(uhat, N, L2OPT)
    pos, wq = _quadrature(n, 8)
    u = evaluate(grid, pos, N, derivatives=False)
    ex = full_fourier_sum(uhat, pos)
    mse = np.sum(wq * (u[:, 0] - ex[:, 0]) ** 2)
    nz = np.nonzero(uhat[0])
    ks = [np.where(nz[d] <= n // 2, nz[d], nz[d] - n) / n for d in range(2)] + [nz[2] / n]
    amp2 = np.abs(uhat[0][nz]) ** 2 * np.where(nz[2] == 0, 1.0, 2.0)
    want = np.sum(amp2 * theory.mode_error_3d(ks, N, L2OPT))
    assert abs(mse - want) < 1e-6 * want


def _band_limited(n, base):
    """Embed the modes of a small half spectrum into a larger grid of size n."""
    nb = base.shape[1]
    out = np.zeros((base.shape[0], n, n, n // 2 + 1), dtype=np.complex128)
    nz = np.nonzero(np.abs(base).sum(axis=0))
    for a, b, c in zip(*nz):
        ka = a if a <= nb // 2 else a - nb
        kb = b if b <= nb // 2 else b - nb
        out[:, ka % n, kb % n, c] = base[:, a, b, c]
    return out


@pytest.mark.parametrize("N", [4, 6])
def test_convergence_order(N):
    base = synth.kolmogorov_spectrum(8, 3, seed=4)           # |k| <= 8/3
    rng = np.random.default_rng(1)
    pos = rng.uniform(0, TWO_PI, size=(3000, 3))
    errs_u, errs_g = [], []
    ns = (16, 32, 64, 128)
    for n in ns:
        uhat = _band_limited(n, base)
        u, g = evaluate(prefilter(uhat, N, L2OPT), pos, N)
        ex, gx = full_fourier_sum(uhat, pos, grad=True)
        errs_u.append(np.sqrt(np.mean((u - ex) ** 2)))
        errs_g.append(np.sqrt(np.mean((g - gx) ** 2)))
    su = np.log2(np.array(errs_u[:-1]) / np.array(errs_u[1:]))
    sg = np.log2(np.array(errs_g[:-1]) / np.array(errs_g[1:]))
    # slopes approach N (value) and N-1 (gradient) from above as kappa -> 0
    assert abs(su[-1] - N) < 0.1 and np.all(su > N - 0.1), su
    assert abs(sg[-1] - (N - 1)) < 0.1 and np.all(sg > N - 1.1), sg
    assert np.all(np.diff(su) < 0) and np.all(np.diff(sg) < 0)


# ---- second derivatives (M^(2) = M D^2) ------------------------------------

def _brute_force_hessian(grid, pos, N, L=TWO_PI):
    from pins import bspline_deriv2_float
    C, n0, n1, n2 = grid.shape
    shape = (n0, n1, n2)
    W, Wd, Wdd = [], [], []
    for d in range(3):
        n = shape[d]
        s = pos[:, d] * (n / L)
        g = np.arange(n)
        w, wd, wdd = (np.zeros((pos.shape[0], n)) for _ in range(3))
        for m in range(-8, 9):
            y = s[:, None] - (g[None, :] + m * n)
            w += bspline_float(N, y)
            wd += bspline_deriv_float(N, y) * (n / L)
            wdd += bspline_deriv2_float(N, y) * (n / L) ** 2
        W.append(w)
        Wd.append(wd)
        Wdd.append(wdd)
    out = []
    for i, j in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)):
        f = list(W)
        if i == j:
            f[i] = Wdd[i]
        else:
            f[i], f[j] = Wd[i], Wd[j]
        out.append(np.einsum("pa,pb,pe,cabe->pc", f[0], f[1], f[2], grid))
    return np.stack(out, axis=-1)


@pytest.mark.parametrize("N", [4, 6])
@pytest.mark.parametrize("shape", [(8, 10, 12), (12, 12, 12)])
def test_hessian_all_lattice_brute_force(N, shape):
    from oracle import evaluate_hessian
    rng = np.random.default_rng(15)
    grid = rng.standard_normal((2,) + shape)
    pos = _edge_positions(rng, 40)
    u, g, h = evaluate_hessian(grid, pos, N)
    u1, g1 = evaluate(grid, pos, N)
    assert np.array_equal(u, u1) or np.max(np.abs(u - u1)) < 1e-13 * np.max(np.abs(grid))
    assert np.max(np.abs(g - g1)) < 1e-12 * np.max(np.abs(grid))
    hb = _brute_force_hessian(grid, pos, N)
    scale = np.max(np.abs(grid)) * (max(shape) / TWO_PI) ** 2
    assert np.max(np.abs(h - hb)) < 1e-11 * scale


@pytest.mark.parametrize("N", [4, 6])
def test_hessian_polynomial_reproduction(N):
    # the grid of test_polynomial_reproduction reproduces s0^a s1^b s2^c
    # exactly, so its second derivatives are reproduced exactly too
    from oracle import evaluate_hessian
    n = 32
    degs = (N - 1, 1, N - 2)
    qs = [_reproducing_coeffs(k, N) for k in degs]
    J = np.arange(n, dtype=np.float64)
    vals = [sum(c * J ** m for m, c in enumerate(q)) for q in qs]
    grid = np.einsum("a,b,e->abe", vals[0], vals[1], vals[2])[None]
    h = TWO_PI / n
    pos = np.random.default_rng(19).uniform(N * h, (n - N) * h, size=(200, 3))
    _, _, hess = evaluate_hessian(grid, pos, N)
    s = pos / h

    def mono(d0, d1, d2):
        out = np.ones(pos.shape[0])
        for ax, dd in enumerate((d0, d1, d2)):
            k = degs[ax]
            coef = 1.0
            for r in range(dd):
                coef *= (k - r)
            out = out * (coef * s[:, ax] ** (k - dd) if k >= dd else 0.0)
        return out / h ** (d0 + d1 + d2)

    exact = np.stack([mono(2, 0, 0), mono(1, 1, 0), mono(1, 0, 1), mono(0, 2, 0), mono(0, 1, 1),
                      mono(0, 0, 2)], axis=-1)
    scale = np.abs(exact).max()          # d2/ds1^2 of s1^1 is exactly zero
    for m in range(6):
        assert np.max(np.abs(hess[:, 0, m] - exact[:, m])) < 1e-12 * scale, m
    assert np.abs(exact[:, 3]).max() == 0.0 and np.abs(exact[:, 0]).max() > 0.0
