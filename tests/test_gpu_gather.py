"""GPU evaluation (gather + contraction) against the oracle, on the oracle's grid.

The coefficient grid is the oracle's FP64 prefilter output loaded through
bsi_field_set_coefficients, which isolates the evaluation from the FFT.  For
FP32 / BF16 storage the oracle evaluates the grid rounded the same way, so the
comparison measures the evaluation arithmetic alone; the end-to-end tests
compare against the unrounded FP64 oracle.
"""
import numpy as np
import pytest

import synth
from gpu_common import log, dev, host, rel_err, bf16_round, edge_positions, TOL_F64, TOL_F32

pytestmark = pytest.mark.gpu

CASES = [
    # n, C, N, coef
    (32, 1, 4, "f64"),
    (32, 3, 4, "f64"),
    (24, 3, 6, "f64"),
    (32, 3, 4, "f32"),
    (48, 3, 6, "f32"),
    (32, 1, 6, "f32"),
    (16, 3, 4, "bf16"),
    (36, 3, 6, "bf16"),
    (32, 1, 4, "bf16"),
    (32, 1, 6, "bf16"),
]


@pytest.fixture(scope="module")
def ctx():
    from paper_1201_4060_amd import Context
    c = Context(0)
    yield c
    c.close()


def _grid(n, C, N, seed):
    from oracle import prefilter
    return prefilter(synth.kolmogorov_spectrum(n, C, seed=seed), N)


@pytest.mark.parametrize("n,C,N,coef", CASES)
def test_gather_matches_oracle(ctx, n, C, N, coef):
    import paper_1201_4060_amd as bsi
    from oracle import evaluate
    log(f"gather n={n} C={C} N={N} coef={coef}")
    dt = {"f64": bsi.BSI_F64, "f32": bsi.BSI_F32, "bf16": bsi.BSI_BF16}[coef]
    grid = _grid(n, C, N, seed=n + C + N)
    pos = np.concatenate([synth.uniform_positions(3001, seed=7),
                          np.random.default_rng(3).uniform(-20, 20, size=(257, 3)),
                          edge_positions()])
    stored = grid if coef == "f64" else (grid.astype(np.float32).astype(np.float64)
                                         if coef == "f32" else bf16_round(grid))
    want_u, want_g = evaluate(stored, pos, N)
    tol = TOL_F64 if coef == "f64" else TOL_F32
    with bsi.Field(ctx, n, C, N, dt) as f:
        f.set_coefficients(dev(grid))
        back = host(f.get_coefficients())
        assert np.array_equal(back, stored)
        for cfg in (None, (0, 256, 0, 0), (4, 128, 1, 0), (8, 64, 1, 0), (2, 192, 0, 0),
                    (6, 256, 1, 0), (12, 128, 1, 0), (8, 256, 1, 1), (16, 256, 1, 0), (8, 256, 1, 0, 256)):
            c = None
            if cfg is not None:
                c = bsi.EvalConfig(sort_tile=cfg[0], block=cfg[1], xcd_remap=cfg[2], variant=cfg[3],
                                   tile_block=cfg[4] if len(cfg) > 4 else 0)
            u, g = f.eval(dev(pos), cfg=c)
            u, g = host(u), host(g)
            eu, eg = rel_err(u, want_u), rel_err(g, want_g)
            log(f"  cfg={cfg} max rel err u={eu.max():.3e} grad={eg.max():.3e}")
            assert eu.max() < tol and eg.max() < tol
            # value only
            u2, _ = f.eval(dev(pos), grad=False, cfg=c)
            assert np.array_equal(host(u2), u)


def test_gather_results_independent_of_tuning(ctx):
    import paper_1201_4060_amd as bsi
    grid = _grid(32, 3, 6, seed=5)
    pos = synth.clustered_positions(20000, 20, 500, 0.1, seed=4)
    with bsi.Field(ctx, 32, 3, 6, bsi.BSI_F32) as f:
        f.set_coefficients(dev(grid))
        ref = None
        for tile in (0, 1, 2, 4, 6, 8, 10, 12, 16, 32):
            for block, variant, tb, ir, remap in ((64, 0, 0, 0, 1), (256, 0, 0, 1, 0), (128, 1, 0, 0, 1),
                                                  (256, 0, 256, 3, 1)):
                u, g = f.eval(dev(pos), cfg=bsi.EvalConfig(sort_tile=tile, block=block, xcd_remap=remap,
                                                           variant=variant, tile_block=tb, item_rounds=ir))
                cur = (host(u), host(g))
                if ref is None:
                    ref = cur
                assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1])


def test_gather_crowded_bucket(ctx):
    # 1e5 particles on one point (one bucket: one coarse range cut into ~50
    # chunks, every per-key atomic on the same key) among a few scattered
    # ones and some non-finite ones: every configuration gives the same bits,
    # and the crowded point matches the oracle
    import paper_1201_4060_amd as bsi
    from oracle import evaluate
    grid = _grid(32, 3, 6, seed=21)
    x0 = np.array([[1.2345, 4.5678, 0.4321]])
    pos = np.concatenate([np.repeat(x0, 100000, axis=0), synth.uniform_positions(5000, seed=22),
                          np.array([[np.nan, 1.0, 1.0]] * 7)])
    perm = np.random.default_rng(23).permutation(pos.shape[0])
    pos = pos[perm]
    want_u, want_g = evaluate(grid, np.concatenate([x0, pos[np.isfinite(pos).all(axis=1)][:200]]), 6)
    with bsi.Field(ctx, 32, 3, 6, bsi.BSI_F64) as f:
        f.set_coefficients(dev(grid))
        ref = None
        # the crowded tile is cut into work items of 1 .. 16 rounds
        for tile, variant, ir in ((8, 0, 0), (8, 0, 1), (8, 0, 16), (4, 0, 2), (8, 1, 0), (0, 1, 0), (2, 1, 0)):
            log(f"  crowded: tile {tile} variant {variant} item rounds {ir}")
            before = f.nonfinite_count()
            u, g = f.eval(dev(pos), cfg=bsi.EvalConfig(sort_tile=tile, block=256, xcd_remap=1,
                                                       variant=variant, item_rounds=ir))
            u, g = host(u), host(g)
            assert f.nonfinite_count() - before == 7
            if ref is None:
                ref = (u, g)
                fin = np.isfinite(pos).all(axis=1)
                assert np.isnan(u[~fin]).all() and np.isnan(g[~fin]).all()
                crowd = np.nonzero((pos == x0).all(axis=1))[0]
                assert crowd.size == 100000
                assert (u[crowd] == u[crowd[0]]).all() and (g[crowd] == g[crowd[0]]).all()
                got_u = np.concatenate([u[crowd[:1]], u[fin][:200]])
                got_g = np.concatenate([g[crowd[:1]], g[fin][:200]])
                assert rel_err(got_u, want_u).max() < TOL_F64
                assert rel_err(got_g, want_g).max() < TOL_F64
            assert np.array_equal(u, ref[0], equal_nan=True) and np.array_equal(g, ref[1], equal_nan=True)


def test_gather_sizes_and_nonfinite(ctx):
    import torch
    import paper_1201_4060_amd as bsi
    from oracle import evaluate
    grid = _grid(16, 3, 4, seed=2)
    with bsi.Field(ctx, 16, 3, 4, bsi.BSI_F64) as f:
        f.set_coefficients(dev(grid))
        for P in (0, 1, 63, 64, 65, 255, 256, 257, 1000):
            pos = synth.uniform_positions(P, seed=P)
            u, g = f.eval(dev(pos.reshape(P, 3)) if P else torch.empty((0, 3), dtype=torch.float64,
                                                                          device="cuda"))
            if P:
                wu, wg = evaluate(grid, pos, 4)
                assert rel_err(host(u), wu).max() < TOL_F64
                assert rel_err(host(g), wg).max() < TOL_F64
        before = f.nonfinite_count()
        pos = np.array([[np.nan, 1, 1], [1, 1, 1], [1, np.inf, 2], [1.7e308, 0, 0]])
        u, g = f.eval(dev(pos))
        u, g = host(u), host(g)
        assert np.isnan(u[[0, 2, 3]]).all() and np.isnan(g[[0, 2, 3]]).all()
        assert np.isfinite(u[1]).all()
        assert f.nonfinite_count() - before == 3


def test_eval_rejects_bad_arguments(ctx):
    import torch
    import paper_1201_4060_amd as bsi
    from paper_1201_4060_amd import _bsi
    with bsi.Field(ctx, 16, 1, 4, bsi.BSI_F32) as f:
        pos = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
        u = torch.zeros((4, 1), dtype=torch.float32, device="cuda")
        with pytest.raises(bsi.BsiError):
            _bsi.bsi_eval(f.handle, pos, -1, u)
        with pytest.raises(bsi.BsiError):
            _bsi.bsi_eval(f.handle, None, 4, u)
        host_pos = torch.zeros((4, 3), dtype=torch.float64)
        with pytest.raises(bsi.BsiError):
            _bsi.bsi_eval(f.handle, host_pos, 4, u)
        with pytest.raises(bsi.BsiError):
            f.eval(pos, cfg=bsi.EvalConfig(sort_tile=8, block=256, xcd_remap=1, tile_block=128))
    for bad in (dict(order=5), dict(order=8), dict(n=(30, 32, 32)), dict(n=(10, 32, 32)),
                dict(ncomp=2), dict(n=(2048, 32, 32))):
        kw = dict(n=(32, 32, 32), ncomp=1, order=4)
        kw.update(bad)
        with pytest.raises(bsi.BsiError):
            bsi.Field(ctx, kw["n"], kw["ncomp"], kw["order"], bsi.BSI_F32)
