"""Synthetic Kolmogorov-spectrum fields in the real-FFT half-spectrum layout.

The spectrum stands in for a snapshot of a dealiased pseudo-spectral DNS:

* Fourier-series coefficients u(x) = sum_k uhat_k exp(i k.x) on [0, 2pi)^3,
  stored as uhat[c][k0][k1][k2] with k0, k1 in [0, n) (signed k' = k or k - n)
  and k2 in [0, n/2] -- the shape numpy's ``rfftn`` produces for a real field.
* Deterministic amplitude |k|^(-11/6), i.e. |uhat|^2 ~ k^(-11/3) (a k^(-5/3)
  energy spectrum), uniform random phase from counter-based SplitMix64.
* Spherical cut-off: every mode with |k| > n/3 is zero, and so is k = 0.
  (k_max dx = 1/3 per direction is the 2/3 dealiasing rule.)
* Exactly Hermitian in the k2 = 0 plane: uhat(-k0, -k1, 0) = conj(uhat(k0, k1, 0)).
  The cut-off keeps every Nyquist index empty, so no other plane needs pairing.
* Three components are projected divergence free, uhat <- (I - k k^T/|k|^2) uhat,
  per mode; the projection is real and even in k, so it keeps the pairing.
* One global factor scales the field so that the mean over components of the
  RMS^2 (sum over the full Hermitian spectrum of |uhat|^2) equals 1.
"""
import numpy as np

from .rng import keyed_uniform


def _signed(idx, n):
    return np.where(idx <= n // 2, idx, idx - n)


def spectrum_nonzero_count(n):
    """Number of half-spectrum entries with 0 < |k| <= n/3 (for documentation/tests)."""
    kc = n // 3
    k = np.arange(-kc, kc + 1)
    k0, k1, k2 = np.meshgrid(k, k, np.arange(0, kc + 1), indexing="ij")
    r2 = k0 * k0 + k1 * k1 + k2 * k2
    return int(np.count_nonzero((9 * r2 <= n * n) & (r2 > 0)))


def kolmogorov_spectrum(n, ncomp, seed, divergence_free=None, out=None):
    """Return uhat[ncomp][n][n][n//2+1] complex128 (see module docstring).

    Random stream c draws the phases of component c; the counter of a mode is
    its flat index in the half-spectrum array (the canonical member of a
    Hermitian pair for the k2 = 0 plane).
    """
    if n % 2:
        raise ValueError("n must be even")
    if ncomp not in (1, 3):
        raise ValueError("ncomp must be 1 or 3")
    if divergence_free is None:
        divergence_free = ncomp == 3
    h = n // 2 + 1
    if out is None:
        out = np.zeros((ncomp, n, n, h), dtype=np.complex128)
    else:
        out[...] = 0
    kc = n // 3
    k1s = np.arange(-kc, kc + 1, dtype=np.int64)
    k2s = np.arange(0, kc + 1, dtype=np.int64)
    K1, K2 = np.meshgrid(k1s, k2s, indexing="ij")
    energy = 0.0
    for k0 in range(-kc, kc + 1):
        r2 = k0 * k0 + K1 * K1 + K2 * K2
        mask = (9 * r2 <= n * n) & (r2 > 0)
        if not mask.any():
            continue
        a1 = K1[mask]
        a2 = K2[mask]
        rr = r2[mask].astype(np.float64)
        amp = rr ** (-11.0 / 12.0)          # |k|^(-11/6)
        # canonical member of the Hermitian pair (only matters for k2 == 0)
        noncanon = (a2 == 0) & ((k0 < 0) | ((k0 == 0) & (a1 < 0)))
        c0 = np.where(noncanon, -k0, k0)
        c1 = np.where(noncanon, -a1, a1)
        counter = ((c0 % n) * n + (c1 % n)) * h + a2
        sgn = np.where(noncanon, -1.0, 1.0)
        vals = np.empty((ncomp, amp.size), dtype=np.complex128)
        for c in range(ncomp):
            theta = 2.0 * np.pi * keyed_uniform(seed, c, counter)
            vals[c] = amp * np.exp(1j * sgn * theta)
        if divergence_free:
            kv = np.stack([np.full(a1.shape, float(k0)), a1.astype(np.float64),
                           a2.astype(np.float64)])
            kdotu = (kv * vals).sum(axis=0)
            vals = vals - kv * (kdotu / rr)
        wgt = np.where(a2 == 0, 1.0, 2.0)
        energy += float((wgt * (np.abs(vals) ** 2)).sum())
        out[:, k0 % n, a1 % n, a2] = vals
    scale = np.sqrt(ncomp / energy)
    out *= scale
    return out
