"""Closed-form per-mode interpolation errors (Section 5).  Test infrastructure only.

For an interpolation written as the convolution u~ = (u D) * C, the interpolant
of one Fourier mode of dimensionless wave number kappa holds the aliases
kappa + i with weights F[C](kappa + i).  The relative squared L2 error of that
mode is
    (F[C](kappa) - 1)^2 + sum_{i != 0} F[C](kappa + i)^2,
and for the l-th derivative the alias terms carry ((kappa + i)/kappa)^(2l).
For the B-spline method the convolution function is c(kappa) B_(N), so
F[C](kappa + i) = c(kappa) sinc^N(kappa + i) (c is a per-mode constant).

Three dimensions (Section 5 says: multiply the 1D components).  The 3D mode's
aliases are the products of the 1D aliases, a_{d,i} = c(kappa_d) sinc^N(kappa_d + i),
so the relative squared error is
    prod_d S_d - 2 prod_d a_{d,0} + 1,    S_d = sum_i a_{d,i}^2,
and for d/dx_d one replaces S_d by sum_i ((kappa_d + i)/kappa_d)^2 a_{d,i}^2.
By the orthogonality corollary of Section 5, the mean-square error of a
multi-mode field is the |uhat|^2-weighted sum of these.
"""
import numpy as np

from .symbol import sinc_power_sum, INTERP, L2OPT

ALIAS_TERMS = 2000


def c_value(kappa, N, variant=L2OPT, terms=20000):
    """c(kappa) of Section 7 for arbitrary (not only grid) kappa."""
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
    if variant == INTERP:
        return 1.0 / sinc_power_sum(kappa, N, terms)
    if variant == L2OPT:
        return np.sinc(kappa) ** N / sinc_power_sum(kappa, 2 * N, terms)
    raise ValueError(variant)


def _alias_weights(kappa, N, variant, terms):
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
    i = np.arange(-terms, terms + 1, dtype=np.float64)
    c = c_value(kappa, N, variant)
    a = c[:, None] * np.sinc(kappa[:, None] + i[None, :]) ** N
    return kappa, i, a


def mode_error_1d(kappa, N, variant=L2OPT, l=0, terms=ALIAS_TERMS):
    """Relative squared L2 error of one mode (Section 5), l-th derivative."""
    kappa, i, a = _alias_weights(kappa, N, variant, terms)
    zero = i == 0
    err = (a[:, zero][:, 0] - 1.0) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = ((kappa[:, None] + i[None, :]) / kappa[:, None]) ** (2 * l)
    alias = np.where(zero[None, :], 0.0, ratio * a * a)
    err = err + alias.sum(axis=1)
    return np.where(kappa == 0.0, 0.0, err)


def mode_error_3d(kappas, N, variant=L2OPT, deriv_axis=None, terms=ALIAS_TERMS):
    """Relative squared L2 error of the 3D mode kappas = (k0, k1, k2) (arrays).

    deriv_axis=None gives the error of the value; deriv_axis=d the error of
    d/dx_d.  Product form of the 1D alias weights (see module doc).
    """
    ks = [np.atleast_1d(np.asarray(k, dtype=np.float64)) for k in kappas]
    S = []
    a0 = []
    for d in range(3):
        kap, i, a = _alias_weights(ks[d], N, variant, terms)
        a0.append(a[:, i == 0][:, 0])
        if deriv_axis == d:
            with np.errstate(divide="ignore", invalid="ignore"):
                ratio = ((kap[:, None] + i[None, :]) / kap[:, None]) ** 2
            ratio = np.where(kap[:, None] == 0.0, np.where(i[None, :] == 0, 1.0, 0.0), ratio)
            S.append((ratio * a * a).sum(axis=1))
        else:
            S.append((a * a).sum(axis=1))
    return S[0] * S[1] * S[2] - 2.0 * a0[0] * a0[1] * a0[2] + 1.0
