"""The seeded workload generator: determinism and the properties the inputs promise."""
import numpy as np

import synth
from synth.rng import splitmix64_mix, GAMMA


def test_splitmix64_reference_output():
    # first output of SplitMix64 started from state 0 (published generator)
    assert int(splitmix64_mix(np.array([GAMMA], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF


def test_keyed_streams_are_deterministic_and_distinct():
    a = synth.keyed_u64(5, 0, np.arange(10))
    b = synth.keyed_u64(5, 0, np.arange(10))
    c = synth.keyed_u64(5, 1, np.arange(10))
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    u = synth.keyed_uniform(1, 2, np.arange(100000))
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01


def _full_from_half(uhat):
    C, n, _, h = uhat.shape
    full = np.zeros((C, n, n, n), dtype=np.complex128)
    full[..., :h] = uhat
    for k2 in range(1, n - h + 1):
        src = uhat[..., k2]
        full[..., n - k2] = np.conj(np.roll(np.flip(src, axis=(1, 2)), 1, axis=(1, 2)))
    return full


def test_kolmogorov_spectrum_properties():
    n = 24
    uhat = synth.kolmogorov_spectrum(n, 3, seed=9)
    assert uhat.shape == (3, n, n, n // 2 + 1)
    k = np.fft.fftfreq(n, 1.0 / n)
    K0, K1, K2 = np.meshgrid(k, k, np.arange(n // 2 + 1), indexing="ij")
    r2 = K0 ** 2 + K1 ** 2 + K2 ** 2
    # cut-off and zero mean
    assert np.all(uhat[:, 9 * r2 > n * n] == 0)
    assert np.all(uhat[:, 0, 0, 0] == 0)
    # divergence free: k . uhat = 0
    div = K0 * uhat[0] + K1 * uhat[1] + K2 * uhat[2]
    assert np.max(np.abs(div)) < 1e-14
    # Hermitian in the k2 = 0 plane
    p = uhat[:, :, :, 0]
    partner = np.conj(np.roll(np.flip(p, axis=(1, 2)), 1, axis=(1, 2)))
    assert np.max(np.abs(p - partner)) == 0.0
    # mean RMS^2 over components is 1 (full Hermitian spectrum)
    full = _full_from_half(uhat)
    assert abs(np.sum(np.abs(full) ** 2) / 3 - 1.0) < 1e-12
    # the field is real
    g = np.fft.ifftn(full, axes=(1, 2, 3), norm="forward")
    assert np.max(np.abs(g.imag)) < 1e-12
    # spectrum slope: amplitude ~ |k|^(-11/6) before projection; scalar field keeps it
    s = synth.kolmogorov_spectrum(n, 1, seed=9)[0]
    m = (r2 > 0) & (9 * r2 <= n * n)
    ratio = np.abs(s[m]) * r2[m] ** (11.0 / 12.0)
    assert np.ptp(ratio) < 1e-12 * ratio.max()


def test_positions():
    p = synth.uniform_positions(1000, 3)
    assert p.shape == (1000, 3) and p.min() >= 0 and p.max() < 2 * np.pi
    assert np.array_equal(p, synth.uniform_positions(1000, 3))
    c = synth.clustered_positions(500, 4, 100, 0.1, seed=2)
    assert c.shape == (900, 3) and c.min() >= 0 and c.max() <= 2 * np.pi
