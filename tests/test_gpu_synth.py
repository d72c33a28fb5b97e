"""The device Kolmogorov generator reproduces the host generator (synth).

Only workloads depend on it (serving and benchmarks at 1024^3, where the host
generator would be slow); the phases come from the same counter-based
SplitMix64 streams, so the two agree to rounding (device sin/cos and the order
of the energy sum differ).
"""
import numpy as np
import pytest

import synth
from gpu_common import log, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,C,seed", [(8, 1, 3), (32, 3, 1), (48, 3, 500), (36, 1, 9)])
def test_device_generator_matches_host(n, C, seed):
    import torch
    import paper_1201_4060_amd as bsi
    want = synth.kolmogorov_spectrum(n, C, seed=seed)
    with bsi.Context(0) as ctx:
        out = torch.empty((C, n, n, n // 2 + 1), dtype=torch.complex128, device="cuda")
        bsi._bsi.bsi_synth_kolmogorov(ctx.handle, n, C, seed, out)
        got = host(out)
        out32 = torch.empty((C, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
        bsi._bsi.bsi_synth_kolmogorov(ctx.handle, n, C, seed, out32)
        got32 = host(out32)
    err = np.abs(got - want).max() / np.abs(want).max()
    log(f"  n={n} C={C}: max |device - host| / max |host| = {err:.2e}")
    assert err < 1e-13
    # modes outside the cut-off are exactly zero on both sides (inside it, the
    # projection can leave an exact zero on one side and a rounding residue on
    # the other)
    kk = np.fft.fftfreq(n, 1.0 / n)
    k2 = np.arange(n // 2 + 1)
    r2 = kk[:, None, None] ** 2 + kk[None, :, None] ** 2 + k2[None, None, :] ** 2
    off = (9 * r2 > n * n) | (r2 == 0)
    assert not np.any(got[:, off]) and not np.any(want[:, off])
    assert np.array_equal(got32, got.astype(np.complex64))
