"""Pins of oracle.prefilter (Section 7: multiply by c(kx)c(ky)c(kz), one inverse FFT).

Pins: a brute-force inverse DFT over the full Hermitian spectrum (tiny grids,
including a non-power-of-two axis); and the interpolation property of the
straightforward choice c = 1/F_D[B_D]: the spline through the coefficients
reproduces the field exactly at the grid nodes, where the field is computed by
direct truncated Fourier summation.
"""
import numpy as np
import pytest

import synth
from oracle import prefilter, prefilter_constants, evaluate, INTERP, L2OPT
from pins import bspline_float, full_fourier_sum


def _random_hermitian_half_spectrum(shape, C, rng):
    """Half spectrum of a random real grid, built by a direct forward DFT."""
    n0, n1, n2 = shape
    g = rng.standard_normal((C, n0, n1, n2))
    e = [np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n) for n in shape]
    full = np.einsum("cxyz,ax,by,dz->cabd", g, e[0], e[1], e[2]) / (n0 * n1 * n2)
    return full[..., : n2 // 2 + 1], full


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 4, 8), (8, 8, 8)])
@pytest.mark.parametrize("N,variant", [(4, L2OPT), (6, INTERP), (4, INTERP)])
def test_against_brute_force_dft(shape, N, variant):
    rng = np.random.default_rng(7)
    C = 2
    half, full = _random_hermitian_half_spectrum(shape, C, rng)
    got = prefilter(half, N, variant)
    c = [prefilter_constants(n, N, variant) for n in shape]
    mult = c[0][:, None, None] * c[1][None, :, None] * c[2][None, None, :]
    e = [np.exp(2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n) for n in shape]
    want = np.einsum("cabd,xa,yb,zd->cxyz", full * mult[None], e[0], e[1], e[2])
    assert np.max(np.abs(want.imag)) < 1e-12
    assert np.max(np.abs(got - want.real)) < 1e-12 * np.max(np.abs(want.real))


@pytest.mark.parametrize("N", [4, 6])
def test_interp_reproduces_field_at_nodes(N):
    n = 16
    uhat = synth.kolmogorov_spectrum(n, 3, seed=11)
    grid = prefilter(uhat, N, INTERP)
    h = 2 * np.pi / n
    g = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), axis=-1).reshape(-1, 3)
    sel = g[:: 7]
    pos = sel * h
    u = evaluate(grid, pos, N, derivatives=False)
    exact = full_fourier_sum(uhat, pos)
    assert np.max(np.abs(u - exact)) < 1e-12 * np.max(np.abs(exact))


@pytest.mark.parametrize("N", [4, 6])
def test_interp_grid_convolved_with_sampled_spline_gives_field(N):
    # u = u_B *_D B_D on the grid (Section 7 discrete model), per axis product
    n = 12
    uhat = synth.kolmogorov_spectrum(n, 1, seed=3)
    ub = prefilter(uhat, N, INTERP)[0]
    nodes = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), axis=-1)
    u_grid = full_fourier_sum(uhat, nodes.reshape(-1, 3) * (2 * np.pi / n))
    u_grid = u_grid[:, 0].reshape(n, n, n)
    r = np.arange(-(N // 2), N // 2 + 1)
    b = bspline_float(N, r.astype(float))
    out = ub
    for axis in range(3):
        acc = np.zeros_like(out)
        for off, wt in zip(r, b):
            acc += wt * np.roll(out, off, axis=axis)
        out = acc
    assert np.max(np.abs(out - u_grid)) < 1e-12 * np.max(np.abs(u_grid))
