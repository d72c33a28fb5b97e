"""Evaluation plans (bsi_eval_plan_*): the binning of the positions and the
gather from it as two calls.  A plan's run is bitwise the one-call evaluation
with the same configuration, also when the binning ran on another stream
while the field's prefilter ran, for several runs over one binning with the
grid changed in between, and after re-binning fewer positions; and within
tolerance of the oracle."""
import numpy as np
import pytest

import synth
from gpu_common import log, dev, host, rel_err, edge_positions, TOL_F32, TOL_F64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1201_4060_amd import Context
    c = Context(0)
    yield c
    c.close()


def _same(a, b):
    return np.array_equal(host(a), host(b), equal_nan=True)


CASES = [  # (n, C, N, coef, basis, cfg)
    (32, 3, 6, "f32", "bspline", (8, 256, 1, 0, 0)),
    (32, 3, 4, "f32", "bspline", (8, 256, 1, 0, 1)),
    (24, 1, 4, "f64", "bspline", (4, 128, 1, 0, 0)),
    (32, 3, 6, "bf16", "bspline", (8, 256, 0, 0, 2)),
    (32, 3, 6, "f32", "bspline", (8, 256, 1, 1, 0)),
    (32, 3, 6, "f32", "bspline", (0, 256, 1, 1, 0)),
    (24, 3, 4, "f32", "lagrange", (8, 256, 1, 0, 0)),
    (24, 3, 4, "f32", "hermite", None),
]


@pytest.mark.parametrize("case", CASES)
def test_plan_equals_one_call(ctx, case):
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate
    n, C, N, coef, basis, cfg = case
    dt = {"f64": bsi.BSI_F64, "f32": bsi.BSI_F32, "bf16": bsi.BSI_BF16}[coef]
    kw = {}
    if basis != "bspline":
        kw = dict(prefilter=bsi.BSI_PREFILTER_NONE,
                  basis=bsi.BSI_BASIS_LAGRANGE if basis == "lagrange" else bsi.BSI_BASIS_HERMITE)
    c = None
    if cfg is not None:
        c = bsi.EvalConfig(sort_tile=cfg[0], block=cfg[1], xcd_remap=cfg[2], variant=cfg[3], item_rounds=cfg[4])
    uhat = synth.kolmogorov_spectrum(n, C, seed=700 + n + N)
    pos = np.concatenate([synth.clustered_positions(3000, 4, 500, 0.2, seed=701), edge_positions(),
                          np.array([[np.nan, 0.5, 0.5]])])
    with bsi.Field(ctx, n, C, N, dt, **kw) as f:
        f.set_spectrum(dev(uhat))
        d = dev(pos)
        u0, g0 = f.eval(d, cfg=c)
        with bsi.EvalPlan(f, pos.shape[0], c) as pl:
            before = f.nonfinite_count()
            pl.bin(d)
            u1, g1 = pl.run()
            assert _same(u0, u1) and _same(g0, g1)
            assert f.nonfinite_count() - before == 1
            u2, _ = pl.run(grad=False)   # a second run over the same binning
            assert _same(u0, u2)
        if basis == "bspline" and coef != "bf16":
            fin = np.isfinite(pos).all(axis=1)
            wu, wg = evaluate(prefilter(uhat, N), pos[fin], N)
            tol = TOL_F64 if coef == "f64" else TOL_F32
            assert rel_err(host(u1)[fin], wu).max() < tol and rel_err(host(g1)[fin], wg).max() < tol


def test_plan_binning_overlaps_the_prefilter(ctx):
    # binning on a side stream while the main stream runs the prefilter; runs
    # over one binning after the grid changed; re-binning fewer positions
    import torch
    import paper_1201_4060_amd as bsi
    n, C, N = 64, 3, 6
    uh1 = dev(synth.kolmogorov_spectrum(n, C, seed=710))
    uh2 = dev(synth.kolmogorov_spectrum(n, C, seed=711))
    pos = dev(synth.clustered_positions(100000, 20, 5000, 0.1, seed=712))
    cfg = bsi.EvalConfig(sort_tile=8, block=256, xcd_remap=1, variant=0)
    with bsi.Field(ctx, n, C, N, bsi.BSI_F32) as f, bsi.EvalPlan(f, pos.shape[0], cfg) as pl:
        main = torch.cuda.current_stream()
        side = torch.cuda.Stream()
        side.wait_stream(main)
        for rep in range(3):
            with torch.cuda.stream(side):
                pl.bin(pos)
            f.set_spectrum(uh1)
            main.wait_stream(side)
            u1, g1 = pl.run()
            torch.cuda.synchronize()
            w1 = f.eval(pos, cfg=cfg)
            assert _same(u1, w1[0]) and _same(g1, w1[1])
        f.set_spectrum(uh2)              # the same binning, a new grid
        u2, g2 = pl.run()
        w2 = f.eval(pos, cfg=cfg)
        torch.cuda.synchronize()
        assert _same(u2, w2[0]) and _same(g2, w2[1])
        assert not _same(u1, u2)
        small = pos[:777].contiguous()   # re-binning fewer positions
        pl.bin(small)
        u3, g3 = pl.run()
        w3 = f.eval(small, cfg=cfg)
        torch.cuda.synchronize()
        assert _same(u3, w3[0]) and _same(g3, w3[1])
        log(f"  plan over {pos.shape[0]} and {small.shape[0]} positions: bitwise equal to one-call evaluation")


def test_plan_errors(ctx):
    import paper_1201_4060_amd as bsi
    from paper_1201_4060_amd import _bsi
    with bsi.Field(ctx, 16, 3, 4, bsi.BSI_F32) as f:
        pos = dev(synth.uniform_positions(100, seed=1))
        with bsi.EvalPlan(f, 50) as pl:
            with pytest.raises(bsi.BsiError) as e:    # run before any binning
                pl._pos = pos
                pl.run()
            assert e.value.status == 1
            with pytest.raises(bsi.BsiError) as e:    # more positions than the plan holds
                pl.bin(pos)
            assert e.value.status == 1
            pl.bin(pos[:50].contiguous())
            u, g = pl.run()
            assert np.isfinite(host(u)).all()
        with pytest.raises(bsi.BsiError):
            _bsi.bsi_eval_plan_create(f.handle, -1)
