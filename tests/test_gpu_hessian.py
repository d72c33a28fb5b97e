"""Second derivatives of the interpolant on the GPU (bsi_eval_hessian) against
the oracle's evaluate_hessian (M^(2) = M D^2, Section 2; tensor product, Section 3).

Tolerances as for u and grad u: per output quantity, max |gpu - oracle| over
the particles relative to max |oracle|, 1e-12 for FP64 grids and arithmetic,
1e-5 for FP32 arithmetic (FP32 and BF16 grids, the oracle evaluated on the
stored coefficients).
"""
import numpy as np
import pytest

import synth
from gpu_common import log, dev, host, rel_err, edge_positions, bf16_round, TOL_F32, TOL_F64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1201_4060_amd import Context
    c = Context(0)
    yield c
    c.close()


def _positions(P, seed):
    return np.concatenate([synth.uniform_positions(P, seed=seed), edge_positions()])


@pytest.mark.parametrize("N", [4, 6])
@pytest.mark.parametrize("C", [1, 3])
def test_hessian_f64(ctx, N, C):
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate_hessian
    n = 32
    grid = prefilter(synth.kolmogorov_spectrum(n, C, seed=40 + C), N)
    pos = _positions(6000, seed=41 + N)
    with bsi.Field(ctx, n, C, N, bsi.BSI_F64) as f:
        f.set_coefficients(dev(grid))
        u, g, h = f.eval_hessian(dev(pos))
        u1, g1 = f.eval(dev(pos))
        u, g, h, u1, g1 = host(u), host(g), host(h), host(u1), host(g1)
    wu, wg, wh = evaluate_hessian(grid, pos, N)
    eu, eg, eh = rel_err(u, wu), rel_err(g, wg), rel_err(h, wh)
    log(f"  f64 n={n} C={C} N={N}: max rel err u {eu.max():.2e} grad {eg.max():.2e} hess {eh.max():.2e}")
    assert eu.max() < TOL_F64 and eg.max() < TOL_F64 and eh.max() < TOL_F64
    # u and grad u agree with the evaluation entry point
    assert rel_err(u, u1).max() < 1e-14 and rel_err(g, g1).max() < 1e-13


@pytest.mark.parametrize("coef", ["f32", "bf16"])
@pytest.mark.parametrize("N", [4, 6])
@pytest.mark.parametrize("C", [1, 3])
def test_hessian_f32_bf16(ctx, coef, N, C):
    # 48^3 grid, 8000 uniform particles: about 37 per 8^3 tile, so tiles of
    # at most 32 particles (two lanes per particle) and larger ones (one lane)
    # both occur
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate_hessian
    n = 48
    grid = prefilter(synth.kolmogorov_spectrum(n, C, seed=50 + C), N)
    stored = grid.astype(np.float32).astype(np.float64) if coef == "f32" else bf16_round(grid)
    pos = _positions(8000, seed=51 + N)
    dt = bsi.BSI_F32 if coef == "f32" else bsi.BSI_BF16
    with bsi.Field(ctx, n, C, N, dt) as f:
        f.set_coefficients(dev(grid))
        u, g, h = f.eval_hessian(dev(pos))
        u, g, h = host(u), host(g), host(h)
    wu, wg, wh = evaluate_hessian(stored, pos, N)
    eu, eg, eh = rel_err(u, wu), rel_err(g, wg), rel_err(h, wh)
    log(f"  {coef} n={n} C={C} N={N}: max rel err u {eu.max():.2e} grad {eg.max():.2e} hess {eh.max():.2e}")
    assert eu.max() < TOL_F32 and eg.max() < TOL_F32 and eh.max() < TOL_F32


def test_hessian_nonfinite_empty_and_no_grad(ctx):
    import torch
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate_hessian
    n, C, N = 16, 3, 4
    grid = prefilter(synth.kolmogorov_spectrum(n, C, seed=60), N)
    pos = np.concatenate([synth.uniform_positions(100, seed=61), [[np.nan, 0.0, 0.0], [0.0, np.inf, 1.0]]])
    with bsi.Field(ctx, n, C, N, bsi.BSI_F64) as f:
        f.set_coefficients(dev(grid))
        before = f.nonfinite_count()
        u, g, h = f.eval_hessian(dev(pos), grad=False)
        assert g is None
        u, h = host(u), host(h)
        assert f.nonfinite_count() - before == 2
        assert np.isnan(u[-2:]).all() and np.isnan(h[-2:]).all()
        _, _, wh = evaluate_hessian(grid, pos[:-2], N)
        assert rel_err(h[:-2], wh).max() < TOL_F64
        u0, g0, h0 = f.eval_hessian(torch.empty((0, 3), dtype=torch.float64, device="cuda"))
        assert h0.shape == (0, C, 6)
        # more positions without a cell than one work item holds (the bucket
        # of non-finite positions is cut into several items, each counted)
        bad = np.full((700, 3), np.nan)
        bad[::3, 1] = np.inf
        mixed = np.concatenate([bad, synth.uniform_positions(300, seed=62)])
        before = f.nonfinite_count()
        u, g, h = f.eval_hessian(dev(mixed))
        u, g, h = host(u), host(g), host(h)
        assert f.nonfinite_count() - before == 700
        assert np.isnan(u[:700]).all() and np.isnan(g[:700]).all() and np.isnan(h[:700]).all()
        _, _, wh = evaluate_hessian(grid, mixed[700:], N)
        assert rel_err(h[700:], wh).max() < TOL_F64


@pytest.mark.parametrize("N", [4, 6])
def test_hessian_full_size_sampled(ctx, N):
    # 256^3 x3, FP32 grid, orders 4 and 6, 10^6 uniform particles (the Hessian
    # benchmark's workload); the oracle on a sample of the particles
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate_hessian
    n, C = 256, 3
    log(f"hessian 256^3 x3 f32 N={N}, 1e6 particles")
    uhat = synth.kolmogorov_spectrum(n, C, seed=1)
    grid = prefilter(uhat, N)
    pos = synth.uniform_positions(1_000_000, seed=101)
    with bsi.Field(ctx, n, C, N, bsi.BSI_F32) as f:
        f.set_coefficients(dev(grid))
        u, g, h = f.eval_hessian(dev(pos))
        u, g, h = host(u), host(g), host(h)
    assert np.isfinite(h).all()
    sample = np.random.default_rng(7).choice(pos.shape[0], 3000, replace=False)
    wu, wg, wh = evaluate_hessian(grid.astype(np.float32).astype(np.float64), pos[sample], N)
    eu, eg, eh = rel_err(u[sample], wu), rel_err(g[sample], wg), rel_err(h[sample], wh)
    log(f"  sampled max rel err u {eu.max():.2e} grad {eg.max():.2e} hess {eh.max():.2e}")
    assert eu.max() < TOL_F32 and eg.max() < TOL_F32 and eh.max() < TOL_F32
    # the field is divergence free: the trace of grad u is small (logged)
    div = g[:, 0, 0] + g[:, 1, 1] + g[:, 2, 2]
    log(f"  rms div / rms grad = {np.sqrt(np.mean(div ** 2) / np.mean(g ** 2)):.2e}")


@pytest.mark.parametrize("coef", ["f64", "f32"])
def test_hessian_crowded_tile(ctx, coef):
    # one 8^3 tile holding 2e4 particles (a dense cluster) beside sparse ones
    # and non-finite positions: the tile's rounds are shared by several
    # workgroups; every particle against the oracle
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate_hessian
    n, C, N = 32, 3, 4
    grid = prefilter(synth.kolmogorov_spectrum(n, C, seed=70), N)
    rng = np.random.default_rng(71)
    h = 2 * np.pi / n
    crowd = (np.array([8.0, 16.0, 0.0]) + rng.uniform(0, 8, size=(20000, 3))) * h
    pos = np.concatenate([crowd, synth.uniform_positions(3000, seed=72), [[np.nan, 1.0, 2.0]]])
    pos = pos[rng.permutation(pos.shape[0])]
    stored = grid if coef == "f64" else grid.astype(np.float32).astype(np.float64)
    dt = bsi.BSI_F64 if coef == "f64" else bsi.BSI_F32
    tol = TOL_F64 if coef == "f64" else TOL_F32
    with bsi.Field(ctx, n, C, N, dt) as f:
        f.set_coefficients(dev(grid))
        u, g, hs = f.eval_hessian(dev(pos))
        u, g, hs = host(u), host(g), host(hs)
    ok = np.isfinite(pos).all(axis=1)
    assert np.isnan(u[~ok]).all() and np.isnan(hs[~ok]).all()
    wu, wg, wh = evaluate_hessian(stored, pos[ok], N)
    eu, eg, eh = rel_err(u[ok], wu), rel_err(g[ok], wg), rel_err(hs[ok], wh)
    log(f"  crowded {coef}: max rel err u {eu.max():.2e} grad {eg.max():.2e} hess {eh.max():.2e}")
    assert eu.max() < tol and eg.max() < tol and eh.max() < tol
