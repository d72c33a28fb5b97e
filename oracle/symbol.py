"""Prefilter constants c(k).  Test infrastructure only (see package doc).

Section 7 transforms to the B-spline basis by multiplying each Fourier mode
by c(k) with kappa = k dx the dimensionless wave number (kappa = k'/n for the
signed FFT index k' in (-n/2, n/2]).  Two choices are given:

* INTERP ("straightforward"): c = 1 / F_D[B_D](k), which makes the spline pass
  through the grid values;
* L2OPT (the optimal choice the paper proposes): c = F[B](kappa) /
  sum_i F[B](kappa + i)^2, minimising the per-mode L2 error.

With F[B_(1)] = sinc and B_(N) the N-fold convolution of B_(1), F[B_(N)] =
sinc^N, sinc(x) = sin(pi x)/(pi x).  F_D[B_D](k) of the m-periodic sampled
spline equals sum_i sinc^N(kappa + i) (Poisson summation; m >= N).  This module
evaluates those lattice sums by direct truncated summation; the HIP library
evaluates them differently (finite cosine sums over B-spline samples), and the
tests pin this truncated series to that closed form.
"""
import functools

import numpy as np

INTERP = "interp"
L2OPT = "l2opt"
NONE = "none"     # c = 1: the grid holds the field's values (Lagrange, linear, Hermite data)

DEFAULT_TERMS = 20000


def sinc_power_sum(kappa, M, terms=DEFAULT_TERMS):
    """S_M(kappa) = sum_{|i| <= terms} sinc(kappa + i)^M, float64, vectorised."""
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
    out = np.zeros(kappa.shape, dtype=np.float64)
    chunk = 4096
    lo = -terms
    while lo <= terms:
        hi = min(lo + chunk, terms + 1)
        i = np.arange(lo, hi, dtype=np.float64)
        out += (np.sinc(kappa[..., None] + i) ** M).sum(axis=-1)
        lo = hi
    return out


def signed_kappa(n):
    """kappa = k'/n for FFT index k = 0..n-1 (k' = k for k <= n/2 else k - n)."""
    k = np.arange(n)
    ks = np.where(k <= n // 2, k, k - n)
    return ks.astype(np.float64) / float(n)


def prefilter_constants(n, N, variant=L2OPT, terms=DEFAULT_TERMS):
    """c(k) for FFT indices k = 0..n-1 of an axis with n points (Section 7)."""
    return _constants(int(n), int(N), variant, int(terms)).copy()


@functools.lru_cache(maxsize=64)
def _constants(n, N, variant, terms):
    # a pure function of its arguments, kept so that repeated prefilters of
    # the same grid size do not re-sum the lattice series
    kappa = signed_kappa(n)
    if variant == NONE:
        return np.ones(n)
    if variant == INTERP:
        return 1.0 / sinc_power_sum(kappa, N, terms)
    if variant == L2OPT:
        return np.sinc(kappa) ** N / sinc_power_sum(kappa, 2 * N, terms)
    raise ValueError(f"unknown variant {variant!r}")
