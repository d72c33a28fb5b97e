"""Closed-form per-mode interpolation errors (Sections 5, 6 and 8).  Test infrastructure only.

Section 5 writes a stencil interpolation as u~ = (u D) * C: the samples of u
times a train of deltas, convolved with the kernel C that the method's matrix
defines piece by piece, C_j(x + N/2 - j) = sum_i M_{j,i} x^(i-1) on [0, 1).
For one Fourier mode phi_kappa the interpolant holds the aliases kappa + i with
weights F[C](kappa + i), F the continuous Fourier transform, and the relative
squared L2 error of the mode is (eq. l2-error)

    |F[C](kappa) - 1|^2 + sum_{i != 0} |F[C](kappa + i)|^2,

for the l-th derivative with the alias terms weighted by ((kappa + i)/kappa)^(2l)
(eq. l2-error-der).  The methods:

* B-spline (Section 7): C = c(kappa) B_(N), c the prefilter constant of the mode
  (``symbol``), B_(N) the kernel of M_(N).
* Lagrange and linear (Section 8): C the kernel of ``methods.lagrange_matrix``.
* Hermite (Section 6, eq. her-int-1): several kernels C_l, one per derivative
  order l - 1 of the data, C_l(x) = C_{0,l}(x) + C_{1,l}(x) with
  C_{j,l}(x - j) = sum_i M_{l + j N/2, i} x^(i-1) on [0, 1); for the mode the
  combined kernel is sum_l (2 pi i kappa)^(l-1) C_l.

The alias series are summed over |i| <= 20000 with the transforms of the
piecewise polynomial kernels in closed form, and cross-checked against the
exact sum by Poisson summation (a reading: the paper gives the series only):
for kernels f, g of compact support,
    sum_i F[f](k + i) conj F[g](k + i) = sum_n R(n) exp(-2 pi i k n),
    R(n) = integral f(y) g(y - n) dy,
and (k + i)^(2l) |F[f](k + i)|^2 = |F[f^(l)](k + i)|^2 / (2 pi)^(2l), which is
finite only when the kernel is C^(l-1) (otherwise f^(l) holds delta functions
and the error is infinite).  ``mode_error_1d`` keeps the paper's series for the
B-spline with F[B_(N)] = sinc^N written out.

Three dimensions (Section 5: multiply the 1D components): the 3D mode's aliases
are products of 1D aliases a_{d,i}, so the relative squared error is
    prod_d S_d - 2 Re prod_d a_{d,0} + 1,    S_d = sum_i |a_{d,i}|^2,
and for d/dx_d, S_d carries ((kappa_d + i)/kappa_d)^2.  By the orthogonality
corollary of Section 5, the mean-square error of a multi-mode field is the
|uhat|^2-weighted sum of these.
"""
from fractions import Fraction

import numpy as np

from .bspline import bspline_matrix
from .methods import lagrange_matrix, hermite_matrix
from .symbol import sinc_power_sum, INTERP, L2OPT, NONE

ALIAS_TERMS = 2000


# ------------------------------------------------ truncated series (B-spline) ---

def c_value(kappa, N, variant=L2OPT, terms=20000):
    """c(kappa) of Section 7 for arbitrary (not only grid) kappa."""
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
    if variant == INTERP:
        return 1.0 / sinc_power_sum(kappa, N, terms)
    if variant == L2OPT:
        return np.sinc(kappa) ** N / sinc_power_sum(kappa, 2 * N, terms)
    if variant == NONE:
        return np.ones_like(kappa)
    raise ValueError(variant)


def _alias_weights(kappa, N, variant, terms):
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
    i = np.arange(-terms, terms + 1, dtype=np.float64)
    c = c_value(kappa, N, variant)
    a = c[:, None] * np.sinc(kappa[:, None] + i[None, :]) ** N
    return kappa, i, a


def mode_error_1d(kappa, N, variant=L2OPT, l=0, terms=ALIAS_TERMS):
    """B-spline: relative squared L2 error of one mode (Section 5), l-th
    derivative, by the truncated alias series with F[B_(N)] = sinc^N."""
    kappa, i, a = _alias_weights(kappa, N, variant, terms)
    zero = i == 0
    err = (a[:, zero][:, 0] - 1.0) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = ((kappa[:, None] + i[None, :]) / kappa[:, None]) ** (2 * l)
    alias = np.where(zero[None, :], 0.0, ratio * a * a)
    err = err + alias.sum(axis=1)
    return np.where(kappa == 0.0, 0.0, err)


# ------------------------------------------------------- piecewise kernels ---

class Kernel:
    """Piecewise polynomial kernel on unit intervals: pieces[a] holds the
    ascending coefficients (exact Fractions) of the polynomial in the local
    variable t = y - a on [a, a + 1); zero outside the listed intervals."""

    def __init__(self, pieces):
        self.pieces = {int(a): [Fraction(c) for c in p] for a, p in pieces.items()}

    def derivative(self):
        return Kernel({a: [(i + 1) * p[i + 1] for i in range(len(p) - 1)] or [Fraction(0)]
                       for a, p in self.pieces.items()})

    def value(self, y):
        """Float evaluation at points y (right-continuous at the knots)."""
        y = np.asarray(y, dtype=np.float64)
        out = np.zeros_like(y)
        a = np.floor(y)
        t = y - a
        for k, p in self.pieces.items():
            m = a == k
            v = np.zeros_like(t[m])
            for c in reversed(p):
                v = v * t[m] + float(c)
            out[m] = v
        return out

    def jumps(self, order):
        """Jump of the order-th derivative at every knot (exact)."""
        k = self
        for _ in range(order):
            k = k.derivative()
        lo = min(k.pieces) if k.pieces else 0
        hi = max(k.pieces) + 1 if k.pieces else 0
        out = {}
        for x in range(lo, hi + 1):
            left = sum(k.pieces[x - 1]) if x - 1 in k.pieces else Fraction(0)   # value at t = 1
            right = k.pieces[x][0] if x in k.pieces else Fraction(0)              # value at t = 0
            out[x] = right - left
        return out

    def continuity(self, max_order=12):
        """Largest p with the kernel C^p (-1 if the kernel itself jumps)."""
        for p in range(max_order + 1):
            if any(v != 0 for v in self.jumps(p).values()):
                return p - 1
        return max_order

    def ft_far(self, k):
        """F[C](k) for |k| >= 1/2 from the jumps of the kernel and its
        derivatives at the knots (integration by parts on every piece):
            F[C](k) = sum_m sum_x [C^(m)](x) exp(-s x) / s^(m+1),  s = 2 pi i k,
        with [C^(m)](x) the exact jump of the m-th derivative at knot x.  Zero
        jumps are exactly zero, so smooth kernels keep their small transforms."""
        k = np.asarray(k, dtype=np.float64)
        s = 2j * np.pi * k
        deg = max(len(p) for p in self.pieces.values())
        out = np.zeros(k.shape, dtype=np.complex128)
        sp = s
        for m in range(deg):
            for x, jump in self.jumps(m).items():
                if jump != 0:
                    out += float(jump) * np.exp(-s * x) / sp
            sp = sp * s
        return out

    def ft(self, k, nodes=48):
        """F[C](k) = integral C(y) exp(-2 pi i k y) dy (Gauss-Legendre per piece;
        exact to rounding for the |k| <= 2 it is used at)."""
        k = np.atleast_1d(np.asarray(k, dtype=np.float64))
        x, w = np.polynomial.legendre.leggauss(nodes)
        t = 0.5 * (x + 1.0)
        w = 0.5 * w
        out = np.zeros(k.shape, dtype=np.complex128)
        for a, p in self.pieces.items():
            vals = np.zeros_like(t)
            for c in reversed(p):
                vals = vals * t + float(c)
            ph = np.exp(-2j * np.pi * k[:, None] * (a + t[None, :]))
            out += (ph * (vals * w)[None, :]).sum(axis=1)
        return out


def _poly_integral_01(p):
    return sum(c / (i + 1) for i, c in enumerate(p))


def _poly_mul(p, q):
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def correlation(f, g, n):
    """R(n) = integral f(y) g(y - n) dy, exact (f, g Kernels, n integer)."""
    acc = Fraction(0)
    for a, p in f.pieces.items():
        b = a - n                      # g's piece on the same unit interval, shifted
        if b in g.pieces:
            acc += _poly_integral_01(_poly_mul(p, g.pieces[b]))
    return acc


def alias_power(f, g, kappa, l=0):
    """sum_i (kappa + i)^(2l) F[f](kappa + i) conj F[g](kappa + i), exact closed
    form by Poisson summation; inf when f or g is not C^(l-1)."""
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
    if l > 0 and (f.continuity() < l - 1 or g.continuity() < l - 1):
        return np.full(kappa.shape, np.inf + 0j)
    fl, gl = f, g
    for _ in range(l):
        fl, gl = fl.derivative(), gl.derivative()
    lo = min(fl.pieces) - max(gl.pieces) - 1
    hi = max(fl.pieces) - min(gl.pieces) + 1
    out = np.zeros(kappa.shape, dtype=np.complex128)
    for n in range(lo, hi + 1):
        r = correlation(fl, gl, n)
        if r != 0:
            out += float(r) * np.exp(-2j * np.pi * kappa * n)
    return out / (2 * np.pi) ** (2 * l)


def kernel_from_matrix(M):
    """Section 5: C_j(x + N/2 - j) = sum_i M_{j,i} x^(i-1) on [0, 1) (1-based j),
    i.e. 0-based row j is the piece on [N/2 - 1 - j, N/2 - j); C = sum_j C_j."""
    N = len(M)
    return Kernel({N // 2 - 1 - j: M[j] for j in range(N)})


def hermite_kernels(N=4):
    """Section 6: C_l = C_{0,l} + C_{1,l}, l = 1..N/2, with C_{j,l}(x - j) =
    sum_i M_{l + j N/2, i} x^(i-1) on [0, 1) -- pieces on [0, 1) and [-1, 0)."""
    M = hermite_matrix(N)
    h = N // 2
    return [Kernel({0: M[l], -1: M[l + h]}) for l in range(h)]


# ------------------------------------------------------------ the methods ---

class Method:
    """A linear interpolation method as kernels K_m with mode-dependent
    weights alpha_m(kappa): the interpolant of phi_kappa is the delta train of
    phi_kappa convolved with sum_m alpha_m(kappa) K_m."""

    def __init__(self, name, kernels, alphas):
        self.name = name
        self.kernels = kernels
        self.alphas = alphas          # callable kappa -> list of arrays

    def alias0(self, kappa):
        kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
        return sum(a * k.ft(kappa) for a, k in zip(self.alphas(kappa), self.kernels))

    def aliases(self, kappa, terms=ALIAS_TERMS):
        """a_i = sum_m alpha_m(kappa) F[K_m](kappa + i) for i = -terms..terms
        ([len(kappa)][2 terms + 1]; |kappa| <= 1/2 so that |kappa + i| >= 1/2
        for i != 0), with the i = 0 column from alias0."""
        kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
        i = np.arange(-terms, terms + 1, dtype=np.float64)
        k = kappa[:, None] + i[None, :]
        kz = np.where(i[None, :] == 0, 1.0, k)       # the i = 0 column is replaced below
        al = self.alphas(kappa)
        out = sum(a[:, None] * km.ft_far(kz) for a, km in zip(al, self.kernels))
        out[:, terms] = self.alias0(kappa)
        return i, out

    def tail(self, kappa, l, terms):
        """sum over |i| > terms of |a_i|^2 ((kappa + i)/kappa)^(2l), to leading
        order: far out a_i = G(kappa) / (2 pi i (kappa + i))^(m+1) with m the
        lowest derivative order with a jump at a knot and
        G = sum_x [sum_q alpha_q K_q^(m)](x) exp(-2 pi i kappa x) (knots are
        integers, so G does not depend on i), and the sum of |kappa + i|^(-p)
        over |i| > terms is two Hurwitz zeta values."""
        from scipy.special import zeta
        kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
        al = self.alphas(kappa)
        deg = max(max(len(p) for p in k.pieces.values()) for k in self.kernels)
        for m in range(deg):
            G = np.zeros(kappa.shape, dtype=np.complex128)
            nz = False
            for a, k in zip(al, self.kernels):
                for x, jump in k.jumps(m).items():
                    if jump != 0:
                        nz = True
                        G += a * float(jump) * np.exp(-2j * np.pi * kappa * x)
            if nz:
                break
        p = 2 * (m + 1) - 2 * l
        if p <= 1:
            return np.full(kappa.shape, np.inf)
        hz = zeta(p, terms + 1 + kappa) + zeta(p, terms + 1 - kappa)
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.abs(G) ** 2 / (2 * np.pi) ** (2 * (m + 1)) * hz / kappa ** (2 * l)

    def alias_sum(self, kappa, l=0):
        """sum_i |a_i|^2 (kappa + i)^(2l), all i, by Poisson summation."""
        kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
        al = self.alphas(kappa)
        out = np.zeros(kappa.shape, dtype=np.complex128)
        for m, km in enumerate(self.kernels):
            for q, kq in enumerate(self.kernels):
                out += al[m] * np.conj(al[q]) * alias_power(km, kq, kappa, l)
        return out.real

    def continuity(self):
        return min(k.continuity() for k in self.kernels)


def bspline_method(N, variant=L2OPT):
    return Method(f"bspline{N}-{variant}", [kernel_from_matrix(bspline_matrix(N))],
                  lambda kap: [c_value(kap, N, variant).astype(np.complex128)])


def lagrange_method(N):
    return Method(f"lagrange{N}" if N > 2 else "linear", [kernel_from_matrix(lagrange_matrix(N))],
                  lambda kap: [np.ones(np.shape(kap), dtype=np.complex128)])


def hermite_method(N=4):
    ks = hermite_kernels(N)
    return Method(f"hermite{N}", ks,
                  lambda kap: [(2j * np.pi * np.asarray(kap, dtype=np.float64)) ** l for l in range(len(ks))])


def mode_error(method, kappa, l=0, terms=20000):
    """Relative squared L2 error of the l-th derivative of one mode (eq.
    l2-error / l2-error-der) for |kappa| <= 1/2: |a_0 - 1|^2 plus the alias
    series over 0 < |i| <= terms (closed-form transforms, so small errors keep
    their relative accuracy) plus its leading-order tail (Method.tail); inf
    when the derivative of the interpolant holds delta functions (kernel not
    C^(l-1)); 0 at kappa = 0."""
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
    if l > 0 and method.continuity() < l - 1:
        return np.where(kappa == 0.0, 0.0, np.inf)
    i, a = method.aliases(kappa, terms)
    zero = i == 0
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = ((kappa[:, None] + i[None, :]) / kappa[:, None]) ** (2 * l)
    alias = np.where(zero[None, :], 0.0, ratio * np.abs(a) ** 2).sum(axis=1)
    err = np.abs(a[:, terms] - 1.0) ** 2 + alias + method.tail(kappa, l, terms)
    return np.where(kappa == 0.0, 0.0, err)


def mode_error_poisson(method, kappa, l=0):
    """The same error with the whole alias series in closed form by Poisson
    summation (exact series, but the i = 0 term is subtracted from it, so
    errors below about 1e-14 lose their relative accuracy)."""
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
    a0 = method.alias0(kappa)
    total = method.alias_sum(kappa, l)
    with np.errstate(divide="ignore", invalid="ignore"):
        err = np.abs(a0 - 1.0) ** 2 - np.abs(a0) ** 2 + total / kappa ** (2 * l)
    return np.where(kappa == 0.0, 0.0, err)


def mode_error_3d(kappas, N, variant=L2OPT, deriv_axis=None, terms=ALIAS_TERMS, method=None):
    # (with a Method the alias series carries its tail term, as in mode_error)
    """Relative squared L2 error of the 3D mode kappas = (k0, k1, k2) (arrays).

    deriv_axis=None gives the error of the value; deriv_axis=d the error of
    d/dx_d.  Product form of the 1D alias weights (see module doc).  With
    method=None the B-spline of order N (prefilter `variant`) by its truncated
    series; otherwise the closed form of that Method.
    """
    ks = [np.atleast_1d(np.asarray(k, dtype=np.float64)) for k in kappas]
    S, a0 = [], []
    for d in range(3):
        if method is None:
            kap, i, a = _alias_weights(ks[d], N, variant, terms)
            a0.append(a[:, i == 0][:, 0].astype(np.complex128))
            if deriv_axis == d:
                with np.errstate(divide="ignore", invalid="ignore"):
                    ratio = ((kap[:, None] + i[None, :]) / kap[:, None]) ** 2
                ratio = np.where(kap[:, None] == 0.0, np.where(i[None, :] == 0, 1.0, 0.0), ratio)
                S.append((ratio * a * a).sum(axis=1))
            else:
                S.append((a * a).sum(axis=1))
        else:
            i, a = method.aliases(ks[d], terms)
            a0.append(a[:, terms])
            p = np.abs(a) ** 2
            if deriv_axis == d:
                with np.errstate(divide="ignore", invalid="ignore"):
                    ratio = ((ks[d][:, None] + i[None, :]) / ks[d][:, None]) ** 2
                ratio = np.where(ks[d][:, None] == 0.0, np.where(i[None, :] == 0, 1.0, 0.0), ratio)
                tail = np.where(ks[d] == 0.0, 0.0, method.tail(ks[d], 1, terms))
                S.append((ratio * p).sum(axis=1) + tail)
            else:
                S.append(p.sum(axis=1) + method.tail(ks[d], 0, terms))
    return S[0] * S[1] * S[2] - 2.0 * (a0[0] * a0[1] * a0[2]).real + 1.0


def figure_curves(kappas, N=4):
    """The per-mode error curves of the comparison (Figs 3 and 4): value, first
    and second derivative of B-spline (both c), Lagrange and Hermite at order N
    and of linear interpolation (N = 2; for the derivatives the paper applies it
    to the derivative fields themselves, whose relative error is its value
    curve).  Returns {method: {l: array}} (inf where a derivative of the
    interpolant holds delta functions)."""
    kappas = np.asarray(kappas, dtype=np.float64)
    methods = [bspline_method(N, L2OPT), bspline_method(N, INTERP), lagrange_method(N), hermite_method(N)]
    out = {m.name: {l: mode_error(m, kappas, l) for l in (0, 1, 2)} for m in methods}
    lin = mode_error(lagrange_method(2), kappas, 0)
    out["linear"] = {0: lin, 1: lin, 2: lin}
    return out
