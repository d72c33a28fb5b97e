"""End to end on the GPU (spectrum in, u and grad u out) against the FP64 oracle.

* the plain method at 32^3, scalar, FP64, order 4, 10^4 uniform particles:
  every particle compared;
* the 256^3 three-component divergence-free field, FP32 grid, orders 4 and 6,
  10^6 uniform particles, in the launch configuration the benchmark times:
  a sample of particles compared against the oracle (which evaluates them one
  by one on the FP64 grid), plus invariants on all of them.
"""
import numpy as np
import pytest

import synth
from gpu_common import log, dev, host, rel_err, TOL_F64, TOL_F32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1201_4060_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("variant", ["l2opt", "interp"])
def test_plain_method_32_f64(ctx, variant):
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate, L2OPT, INTERP
    log(f"end2end 32^3 f64 {variant}")
    v = {"l2opt": (L2OPT, bsi.BSI_PREFILTER_L2OPT), "interp": (INTERP, bsi.BSI_PREFILTER_INTERP)}[variant]
    uhat = synth.kolmogorov_spectrum(32, 1, seed=0)
    pos = synth.uniform_positions(10000, seed=100)
    want_u, want_g = evaluate(prefilter(uhat, 4, v[0]), pos, 4)
    with bsi.Field(ctx, 32, 1, 4, bsi.BSI_F64, prefilter=v[1]) as f:
        f.set_spectrum(dev(uhat))
        u, g = f.eval(dev(pos))
    eu, eg = rel_err(host(u), want_u), rel_err(host(g), want_g)
    log(f"  u {eu.max():.3e} grad {eg.max():.3e}")
    assert eu.max() < TOL_F64 and eg.max() < TOL_F64


@pytest.mark.parametrize("N", [4, 6])
def test_field_256_f32_sampled(ctx, N):
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate
    log(f"end2end 256^3 x3 f32 N={N}")
    uhat = synth.kolmogorov_spectrum(256, 3, seed=1)
    pos = synth.uniform_positions(1000000, seed=101)
    with bsi.Field(ctx, 256, 3, N, bsi.BSI_F32) as f:
        f.set_spectrum(dev(uhat))
        u, g = f.eval(dev(pos))
        u, g = host(u), host(g)
    assert np.isfinite(u).all() and np.isfinite(g).all()
    # divergence free field: trace of the gradient is small relative to |grad|
    div = g[:, 0, 0] + g[:, 1, 1] + g[:, 2, 2]
    log(f"  rms div / rms grad = {np.sqrt(np.mean(div**2) / np.mean(g**2)):.3e}")
    sample = np.random.default_rng(N).choice(pos.shape[0], 4000, replace=False)
    grid = prefilter(uhat, N)
    want_u, want_g = evaluate(grid, pos[sample], N)
    eu, eg = rel_err(u[sample], want_u), rel_err(g[sample], want_g)
    log(f"  sampled max rel err u {eu.max():.3e} grad {eg.max():.3e}")
    assert eu.max() < TOL_F32 and eg.max() < TOL_F32
