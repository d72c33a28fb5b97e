"""GPU prefilter (symbol multiply + inverse 3D real FFT) against the oracle grid."""
import numpy as np
import pytest

import synth
from gpu_common import log, dev, host, TOL_F64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1201_4060_amd import Context
    c = Context(0)
    yield c
    c.close()


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def _random_spectrum(shape, C, rng):
    """Generic (non-Hermitian, full-band) half spectrum: exercises every bin."""
    n0, n1, n2 = shape
    return (rng.standard_normal((C, n0, n1, n2 // 2 + 1))
            + 1j * rng.standard_normal((C, n0, n1, n2 // 2 + 1)))


SIZES = [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256]


@pytest.mark.parametrize("n", SIZES)
def test_prefilter_f64_all_sizes(ctx, n):
    import paper_1201_4060_amd as bsi
    from oracle import prefilter
    log(f"prefilter f64 n={n}")
    N = 4 if n < 12 else 6
    rng = np.random.default_rng(n)
    uhat = _random_spectrum((n, n, n), 1, rng)
    want = prefilter(uhat, N)
    with bsi.Field(ctx, n, 1, N, bsi.BSI_F64) as f:
        f.set_spectrum(dev(uhat))
        got = host(f.get_coefficients())
    err = _rel(got, want)
    log(f"  rel err {err:.3e}")
    assert err < TOL_F64


@pytest.mark.parametrize("shape,C,N,variant", [
    ((32, 48, 64), 3, 4, "l2opt"),
    ((64, 32, 24), 1, 6, "interp"),
    ((16, 16, 96), 3, 6, "l2opt"),
])
def test_prefilter_f64_noncubic(ctx, shape, C, N, variant):
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, INTERP, L2OPT
    log(f"prefilter noncubic {shape} C={C} N={N} {variant}")
    rng = np.random.default_rng(11)
    uhat = _random_spectrum(shape, C, rng)
    v = {"l2opt": (L2OPT, bsi.BSI_PREFILTER_L2OPT), "interp": (INTERP, bsi.BSI_PREFILTER_INTERP)}[variant]
    want = prefilter(uhat, N, v[0])
    with bsi.Field(ctx, shape, C, N, bsi.BSI_F64, prefilter=v[1]) as f:
        f.set_spectrum(dev(uhat))
        got = host(f.get_coefficients())
    assert _rel(got, want) < TOL_F64


@pytest.mark.parametrize("n,C,N", [(64, 3, 4), (192, 3, 6), (256, 1, 6), (384, 1, 4)])
@pytest.mark.parametrize("inprec", ["c128", "c64"])
def test_prefilter_f32(ctx, n, C, N, inprec):
    import paper_1201_4060_amd as bsi
    from oracle import prefilter
    log(f"prefilter f32 n={n} C={C} N={N} in={inprec}")
    uhat = synth.kolmogorov_spectrum(n, C, seed=n)
    if inprec == "c64":
        uhat = uhat.astype(np.complex64)
    want = prefilter(uhat.astype(np.complex128), N)
    with bsi.Field(ctx, n, C, N, bsi.BSI_F32) as f:
        f.set_spectrum(dev(uhat))
        got = host(f.get_coefficients())
    err = _rel(got, want)
    log(f"  rel err {err:.3e}")
    assert err < 2e-6


def test_prefilter_large_f32_sample(ctx):
    # 512^3 and 1024^3 transforms (one component), compared on sampled lines
    import paper_1201_4060_amd as bsi
    import torch
    for n in (512, 768, 1024):
        log(f"prefilter f32 n={n} sampled")
        rng = np.random.default_rng(n)
        uhat_small = synth.kolmogorov_spectrum(16, 1, seed=n)
        # embed a band-limited spectrum so the exact grid is a short Fourier sum
        uhat = torch.zeros((1, n, n, n // 2 + 1), dtype=torch.complex128)
        nz = np.nonzero(uhat_small[0])
        for a, b, c in zip(*nz):
            ka = a if a <= 8 else a - 16
            kb = b if b <= 8 else b - 16
            uhat[0, ka % n, kb % n, c] = complex(uhat_small[0, a, b, c])
        from oracle import prefilter_constants
        with bsi.Field(ctx, n, 1, 4, bsi.BSI_F32) as f:
            f.set_spectrum(uhat.cuda())
            got = f.get_coefficients()
            idx = rng.integers(0, n, size=(64, 3))
            vals = host(got[0, idx[:, 0], idx[:, 1], idx[:, 2]])
        c = prefilter_constants(n, 4)
        want = np.zeros(64)
        for a, b, cc in zip(*nz):
            ka = a if a <= 8 else a - 16
            kb = b if b <= 8 else b - 16
            m = c[ka % n] * c[kb % n] * c[cc] * uhat_small[0, a, b, cc]
            ph = 2 * np.pi * (ka * idx[:, 0] + kb * idx[:, 1] + cc * idx[:, 2]) / n
            w = 1.0 if cc == 0 else 2.0
            want += w * (m * np.exp(1j * ph)).real
        err = np.max(np.abs(vals - want)) / np.max(np.abs(want))
        log(f"  rel err {err:.3e}")
        assert err < 2e-6
        del uhat
        torch.cuda.empty_cache()


def test_prefilter_bf16_is_rne_of_f32(ctx):
    import paper_1201_4060_amd as bsi
    from gpu_common import bf16_round
    n, C, N = 32, 3, 6
    uhat = synth.kolmogorov_spectrum(n, C, seed=1)
    with bsi.Field(ctx, n, C, N, bsi.BSI_F32) as f32, bsi.Field(ctx, n, C, N, bsi.BSI_BF16) as fb:
        f32.set_spectrum(dev(uhat))
        fb.set_spectrum(dev(uhat))
        g32 = host(f32.get_coefficients())
        gb = host(fb.get_coefficients())
    assert np.array_equal(gb, bf16_round(g32))
