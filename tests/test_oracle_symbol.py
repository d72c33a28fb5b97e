"""Pins of oracle.symbol: the prefilter constants c(k) of Section 7.

Pins: c(0) = 1; the oracle's truncated lattice sums against the finite cosine
sums over B-spline samples (Poisson summation); INTERP against a brute-force
DFT of the periodic sampled B-spline B_D as Section 7 defines it; exact values
at kappa = 1/3; evenness; and that the L2-optimal c really minimises the
per-mode error expression of Section 5.
"""
from fractions import Fraction
from math import cos, pi, sin, sqrt

import numpy as np
import pytest

from oracle.symbol import (sinc_power_sum, prefilter_constants, signed_kappa,
                           INTERP, L2OPT)
from oracle import theory
from pins import bspline_exact


def closed_form_S(kappa, M):
    """sum_s B_M(s) cos(2 pi kappa s) over the integers in the support."""
    half = M // 2 + 1
    acc = np.zeros_like(np.asarray(kappa, dtype=np.float64))
    for s in range(-half, half + 1):
        acc = acc + float(bspline_exact(M, s)) * np.cos(2 * np.pi * kappa * s)
    return acc


@pytest.mark.parametrize("N", [2, 4, 6, 8])
@pytest.mark.parametrize("variant", [INTERP, L2OPT])
def test_c_at_zero_is_one(N, variant):
    assert abs(prefilter_constants(16, N, variant)[0] - 1.0) < 1e-15


@pytest.mark.parametrize("M,tol", [(4, 3e-14), (6, 4e-15), (8, 4e-15), (12, 4e-15)])
def test_truncated_series_matches_poisson_closed_form(M, tol):
    kappa = np.linspace(-0.5, 0.5, 101)
    a = sinc_power_sum(kappa, M)
    b = closed_form_S(kappa, M)
    assert np.max(np.abs(a - b) / np.abs(b)) < tol


@pytest.mark.parametrize("N", [4, 6])
@pytest.mark.parametrize("m", [8, 12, 16])
def test_interp_is_inverse_dft_of_sampled_bspline(N, m):
    # Section 7: B_D(x) = B(x) for x < m/2 and B(x - m) otherwise, x = 0..m-1;
    # F_D[f](k) = sum_x f(x) exp(-2 pi i x k / m); INTERP c = 1 / F_D[B_D].
    x = np.arange(m)
    BD = np.array([float(bspline_exact(N, xi if xi < m / 2 else xi - m)) for xi in x])
    k = np.arange(m)
    FD = (BD[None, :] * np.exp(-2j * np.pi * np.outer(k, x) / m)).sum(axis=1)
    assert np.max(np.abs(FD.imag)) < 1e-14
    c = prefilter_constants(m, N, INTERP)
    assert np.max(np.abs(c * FD.real - 1.0)) < 1e-13


def test_exact_values_at_one_third():
    k3 = np.array([1.0 / 3.0])
    # INTERP: S_4(1/3) = 2/3 + 2*(1/6)*cos(2pi/3) = 1/2 -> c = 2
    #         S_6(1/3) = 11/20 - 13/60 - 1/120 = 13/40 -> c = 40/13
    assert abs(theory.c_value(k3, 4, INTERP)[0] - 2.0) < 1e-14
    assert abs(theory.c_value(k3, 6, INTERP)[0] - 40.0 / 13.0) < 1e-14
    # L2OPT: sinc(1/3) = 3 sqrt(3) / (2 pi); S_2N from exact B_2N samples
    sinc13 = 3.0 * sqrt(3.0) / (2.0 * pi)
    for N in (4, 6):
        S2N = sum(float(bspline_exact(2 * N, s)) * cos(2 * pi * s / 3.0)
                  for s in range(-N, N + 1))
        expect = sinc13 ** N / S2N
        assert abs(theory.c_value(k3, N, L2OPT)[0] - expect) < 1e-14 * expect


@pytest.mark.parametrize("N", [4, 6])
@pytest.mark.parametrize("variant", [INTERP, L2OPT])
def test_even_in_kappa(N, variant):
    n = 64
    c = prefilter_constants(n, N, variant)
    k = np.arange(1, n // 2)
    assert np.max(np.abs(c[k] - c[n - k]) / c[k]) < 1e-15


@pytest.mark.parametrize("N", [4, 6])
def test_l2opt_minimises_mode_error(N):
    # per-mode error of Section 5 with F[C](kappa+i) = c sinc^N(kappa+i),
    # written out for a free multiplier c
    kappa = np.linspace(0.02, 0.5, 25)
    i = np.arange(-3000, 3001)
    s = np.sinc(kappa[:, None] + i[None, :]) ** N
    s0 = s[:, i == 0][:, 0]
    alias = (s ** 2).sum(axis=1) - s0 ** 2

    def err(c):
        return (c * s0 - 1.0) ** 2 + c * c * alias

    c_opt = theory.c_value(kappa, N, L2OPT)
    c_int = theory.c_value(kappa, N, INTERP)
    e_opt = err(c_opt)
    assert np.all(e_opt <= err(c_opt * (1 + 1e-3)))
    assert np.all(e_opt <= err(c_opt * (1 - 1e-3)))
    assert np.all(e_opt <= err(c_int) + 1e-16)
    # and theory.mode_error_1d is that same expression
    assert np.allclose(theory.mode_error_1d(kappa, N, L2OPT), e_opt, rtol=1e-9, atol=1e-15)


def test_signed_kappa_layout():
    assert list(signed_kappa(8) * 8) == [0, 1, 2, 3, 4, -3, -2, -1]
