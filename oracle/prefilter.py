"""Prefilter: spectrum -> B-spline coefficient grid.  Test infrastructure only.

Section 7: the B-spline coefficients u_B satisfy u = u_B *_D B_D; in Fourier
space this is F_D[u_B](k) = c(k) F_D[u](k), and in three dimensions the
multiplier is the product c(kx) c(ky) c(kz).  The method statement at the end
of Section 7 then needs one inverse FFT to reach u_B on the grid.

Convention of the spectrum (the paper works on [0, 1] with exp(2 pi i k x); a
field on [0, 2 pi)^3 rescales this): uhat are Fourier-series coefficients,
u(x) = sum_k uhat_k exp(i k.x), held as the real-FFT half spectrum
uhat[c][k0][k1][k2], k2 = 0..n2/2.  Grid values are then the *unnormalised*
inverse DFT of uhat, i.e. numpy's irfftn with norm="forward".  The library FFT
is used as one step; it is checked against a brute-force DFT in the tests.
"""
import numpy as np

from .symbol import prefilter_constants, L2OPT


def prefilter(uhat, N, variant=L2OPT, shape=None):
    """Return the coefficient grid u_B[c][g0][g1][g2] (float64).

    uhat  : complex array [C][n0][n1][n2//2+1]
    N     : spline order
    shape : (n0, n1, n2); n2 defaults to 2*(last dim - 1)
    """
    uhat = np.asarray(uhat)
    if uhat.ndim != 4:
        raise ValueError("uhat must be [C][n0][n1][n2/2+1]")
    if shape is None:
        shape = (uhat.shape[1], uhat.shape[2], 2 * (uhat.shape[3] - 1))
    n0, n1, n2 = shape
    c0 = prefilter_constants(n0, N, variant)
    c1 = prefilter_constants(n1, N, variant)
    c2 = prefilter_constants(n2, N, variant)[: n2 // 2 + 1]
    # 3D multiplier c(k0) c(k1) c(k2) applied to every component, in FP64
    mult = c0[:, None, None] * c1[None, :, None] * c2[None, None, :]
    ub_hat = uhat.astype(np.complex128) * mult[None]
    return np.fft.irfftn(ub_hat, s=(n0, n1, n2), axes=(1, 2, 3), norm="forward")
