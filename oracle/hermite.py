"""Cubic Hermite interpolation of a spectral field in three dimensions.

Test infrastructure only (see package doc).

Section 2 gives the 1D method: on a cell, f = (u(0), u'(0), u(1), u'(1)) and
u~ = f^T M xbar with the printed 4 x 4 matrix M (``methods.hermite_matrix``).
Section 3 builds the 3D method as the tensor product: the local tensor
B = f_z[f_y[f_x[u]]] holds, for each of the 2 x 2 x 2 cell corners, the value
and the mixed derivatives d^(a0+a1+a2) u / dx^a0 dy^a1 dz^a2 with a_d in {0, 1},
and u~ = B x1 (M xbar) x2 (M ybar) x3 (M zbar); a first derivative replaces one
factor by M^(1) = M D.  Section 6 writes the same thing as several convolutions,
one per derivative, which is why the method needs (N/2)^3 = 8 fields per
component, each one inverse FFT (Table 2).

The derivative fields come from the spectrum: in grid units (spacing one, the
Section 5 rescaling) d/ds of exp(2 pi i k' s / n) is i 2 pi k'/n times it, so
field a = irfftn(prod_d (i 2 pi k'_d / n)^(a_d) uhat).  Reading (the paper is
silent): the Nyquist index k' = n/2 of an axis that is differentiated an odd
number of times is set to zero, as in spectral differentiation of real fields.

Cells and offsets follow the same rule as the B-spline evaluation
(``evaluate.cells``): x_j = floor(x) + j, j in {0, 1} (Section 6).
"""
import numpy as np

from .evaluate import cells, inv_spacing, TWO_PI
from .methods import hermite_matrix, hermite_data_rows, to_f64
from .bspline import derivative_matrix

ORDERS = [(a0, a1, a2) for a0 in (0, 1) for a1 in (0, 1) for a2 in (0, 1)]


def derivative_factor(n, a):
    """(i 2 pi k'/n)^a for FFT indices k = 0..n-1 of an axis (complex)."""
    k = np.arange(n)
    ks = np.where(k <= n // 2, k, k - n).astype(np.float64)
    f = (2j * np.pi * ks / n) ** a
    if a % 2 == 1 and n % 2 == 0:
        f[n // 2] = 0.0
    return f


def derivative_grids(uhat, shape=None):
    """The 8 Hermite data fields per component: dict a -> float64 [C][n0][n1][n2]
    with field a = d^(a0+a1+a2) u / ds0^a0 ds1^a1 ds2^a2 on the grid (grid units)."""
    uhat = np.asarray(uhat)
    if shape is None:
        shape = (uhat.shape[1], uhat.shape[2], 2 * (uhat.shape[3] - 1))
    n0, n1, n2 = shape
    out = {}
    for a in ORDERS:
        f0 = derivative_factor(n0, a[0])
        f1 = derivative_factor(n1, a[1])
        f2 = derivative_factor(n2, a[2])[: n2 // 2 + 1]
        mult = f0[:, None, None] * f1[None, :, None] * f2[None, None, :]
        out[a] = np.fft.irfftn(uhat.astype(np.complex128) * mult[None], s=(n0, n1, n2), axes=(1, 2, 3),
                               norm="forward")
    return out


def interleaved(dgrids):
    """The 8 fields as one array [C][2 n0][2 n1][2 n2]: entry (2 g + a) holds field a
    at grid point g (the storage the library's Hermite fields use)."""
    g = dgrids[(0, 0, 0)]
    C, n0, n1, n2 = g.shape
    out = np.empty((C, 2 * n0, 2 * n1, 2 * n2))
    for a, v in dgrids.items():
        out[:, a[0]::2, a[1]::2, a[2]::2] = v
    return out


def _weights(t, inv_h):
    """Hermite weights h[P][4] (data order of Section 2) and their derivative."""
    M = hermite_matrix(4)
    Mf = to_f64(M)
    M1 = to_f64(derivative_matrix(M, 1))
    powers = np.stack([t ** i for i in range(4)], axis=-1)
    return powers @ Mf.T, (powers @ M1.T) * inv_h


def evaluate_hermite(dgrids, pos, lengths=(TWO_PI, TWO_PI, TWO_PI)):
    """u [P][C] and grad [P][C][3] of the 3D cubic Hermite interpolant.

    dgrids: the dict of ``derivative_grids``.  Plain sum over the 4^3 entries of
    the local tensor B: entry (r0, r1, r2), r_d = (corner, order) from the
    Section 2 data order, holds field (order_0, order_1, order_2) at grid point
    cell + corner.  Non-finite positions give NaN.
    """
    g0 = dgrids[(0, 0, 0)]
    C, n0, n1, n2 = g0.shape
    shape = (n0, n1, n2)
    pos = np.asarray(pos, dtype=np.float64)
    P = pos.shape[0]
    cell, t, finite = cells(pos, shape, lengths)
    H, Hd = [], []
    for d in range(3):
        h, hd = _weights(t[:, d], inv_spacing(shape[d], lengths[d]))
        H.append(h)
        Hd.append(hd)
    rows = hermite_data_rows(4)
    flat = {a: v.reshape(C, -1) for a, v in dgrids.items()}
    u = np.zeros((P, C))
    grad = np.zeros((P, C, 3))
    for r0, (c0, a0) in enumerate(rows):
        i0 = np.mod(cell[:, 0] + c0, n0)
        for r1, (c1, a1) in enumerate(rows):
            i1 = np.mod(cell[:, 1] + c1, n1)
            for r2, (c2, a2) in enumerate(rows):
                i2 = np.mod(cell[:, 2] + c2, n2)
                vals = flat[(a0, a1, a2)][:, (i0 * n1 + i1) * n2 + i2].T
                r = (r0, r1, r2)
                u += (H[0][:, r0] * H[1][:, r1] * H[2][:, r2])[:, None] * vals
                for d in range(3):
                    f = [H[k][:, r[k]] for k in range(3)]
                    f[d] = Hd[d][:, r[d]]
                    grad[:, :, d] += (f[0] * f[1] * f[2])[:, None] * vals
    if not finite.all():
        u[~finite] = np.nan
        grad[~finite] = np.nan
    return u, grad
