"""Batching form on the GPU: many fields in one persistent gather launch.

Every item of a batch must come out bitwise equal to bsi_eval_ex of its field
with the configuration the planner chose for it (the per-particle arithmetic
is shared), with and without the HIP graph, on every graph replay; parity with
the oracle is checked directly on small fields (grids from the oracle's
prefilter) and inherited elsewhere.
"""
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


def _field(ctx, n, C, N, coef, seed):
    import paper_1201_4060_amd as bsi
    from oracle import prefilter
    grid = prefilter(synth.kolmogorov_spectrum(n, C, seed=seed), N)
    f = bsi.Field(ctx, n, C, N, coef)
    f.set_coefficients(dev(grid))
    return f, grid


def _outputs(f, P, grad=True):
    import torch
    u = torch.full((P, f.ncomp), float("nan"), dtype=f.out_dtype, device="cuda")
    g = torch.full((P, f.ncomp, 3), float("nan"), dtype=f.out_dtype, device="cuda") if grad else None
    return u, g


def _positions(P, seed, clustered):
    """Exactly P positions: uniform, or half uniform and half in a few blobs."""
    if not clustered or P < 8:
        return synth.uniform_positions(P, seed=seed)
    p = synth.clustered_positions(P // 2, 3, (P - P // 2) // 3, 0.2, seed=seed)
    extra = synth.uniform_positions(P - p.shape[0], seed=seed + 7)
    return np.ascontiguousarray(np.concatenate([p, extra]))


def _single(f, pos, cfg, grad=True):
    return f.eval(pos, grad=grad, cfg=cfg)


def _same(a, b):
    return np.array_equal(host(a), host(b), equal_nan=True)


def _cfg(bsi, tile, variant):
    return bsi.EvalConfig(sort_tile=tile, block=256, xcd_remap=1, variant=variant, tiles_per_group=2)


SPECS = [
    # n, C, N, P, (sort_tile, variant) or None for the tuned/default choice
    (32, 3, 4, 20000, (8, 0)),
    (48, 3, 6, 5000, (4, 0)),
    (32, 1, 6, 3000, (8, 1)),
    (64, 3, 6, 1, None),
    (24, 1, 4, 0, None),
    (36, 3, 4, 7777, (6, 0)),
    (64, 3, 4, 40000, (16, 1)),
    (32, 3, 6, 2500, (12, 0)),
    # every (order, components) class with tiled and direct items: each class
    # has a tile kernel and a direct kernel of its own
    (48, 1, 4, 9000, (8, 0)),
    (36, 1, 6, 6000, (8, 0)),
    (24, 1, 4, 5000, (8, 1)),
]


def test_batch_matches_single_and_oracle(ctx):
    import torch
    import paper_1201_4060_amd as bsi
    from oracle import evaluate
    fields, grids, items, cfgs, pos_h = [], [], [], [], []
    for i, (n, C, N, P, cfg) in enumerate(SPECS):
        f, grid = _field(ctx, n, C, N, bsi.BSI_F32, seed=20 + i)
        fields.append(f)
        grids.append(grid)
        p = _positions(P, 40 + i, clustered=True)
        if P >= 100:
            p[:9] = edge_positions()
        pos_h.append(p)
        pos = dev(p)
        u, g = _outputs(f, P)
        items.append((f, pos, u, g))
        cfgs.append(None if cfg is None else _cfg(bsi, *cfg))
    tuned = [c if c is not None else bsi._bsi.bsi_ctx_lookup_config(ctx.handle, f.handle, it[1].shape[0])
             for c, f, it in zip(cfgs, fields, items)]
    try:
        with bsi.Batch(ctx, items, cfgs=tuned) as b:
            for use_graph in (False, True):
                for it in items:
                    it[2].fill_(float("nan"))
                    it[3].fill_(float("nan"))
                b.run(use_graph=use_graph)
                torch.cuda.synchronize()
                for i, (f, pos, u, g) in enumerate(items):
                    planned = b.item_config(i)
                    if pos.shape[0] == 0:
                        continue
                    us, gs = _single(f, pos, planned)
                    torch.cuda.synchronize()
                    log(f"  item {i} graph={use_graph} planned tile={planned.sort_tile} "
                        f"variant={planned.variant} P={pos.shape[0]}")
                    assert _same(u, us) and _same(g, gs), f"item {i} differs from bsi_eval_ex"
            for i, (f, pos, u, g) in enumerate(items):
                P = pos.shape[0]
                if P == 0:
                    continue
                n, C, N = SPECS[i][0], SPECS[i][1], SPECS[i][2]
                stored = grids[i].astype(np.float32).astype(np.float64)
                sel = np.arange(min(P, 800))
                want_u, want_g = evaluate(stored, pos_h[i][sel], N)
                if P >= 100:
                    eu, eg = rel_err(host(u)[sel], want_u), rel_err(host(g)[sel], want_g)
                else:
                    # too few particles for a per-quantity maximum: scale by
                    # the largest value or derivative component instead
                    eu = np.abs(host(u)[sel] - want_u).max() / np.abs(want_u).max()
                    eg = np.abs(host(g)[sel] - want_g).max() / np.abs(want_g).max()
                    eu, eg = np.array([eu]), np.array([eg])
                log(f"  item {i} n={n} C={C} N={N}: rel err u {eu.max():.2e} grad {eg.max():.2e}")
                assert eu.max() < TOL_F32 and eg.max() < TOL_F32
    finally:
        for f in fields:
            f.close()


@pytest.mark.parametrize("coef", ["f64", "bf16"])
def test_batch_other_types(ctx, coef):
    import torch
    import paper_1201_4060_amd as bsi
    dt = {"f64": bsi.BSI_F64, "bf16": bsi.BSI_BF16}[coef]
    specs = [(32, 3, 4, 6000, (8, 0)), (24, 3, 6, 4000, (4, 0)), (32, 1, 6, 3000, (4, 1)),
             (16, 3, 4, 500, (8, 0))]
    fields, items = [], []
    try:
        for i, (n, C, N, P, cfg) in enumerate(specs):
            f, _ = _field(ctx, n, C, N, dt, seed=60 + i)
            fields.append(f)
            pos = dev(synth.uniform_positions(P, seed=70 + i))
            u, g = _outputs(f, P)
            items.append((f, pos, u, g))
        cfgs = [_cfg(bsi, *s[4]) for s in specs]
        with bsi.Batch(ctx, items, cfgs=cfgs) as b:
            b.run(use_graph=True)
            torch.cuda.synchronize()
            for i, (f, pos, u, g) in enumerate(items):
                us, gs = _single(f, pos, b.item_config(i))
                torch.cuda.synchronize()
                log(f"  {coef} item {i}: tile {b.item_config(i).sort_tile} variant {b.item_config(i).variant}")
                assert _same(u, us) and _same(g, gs)
    finally:
        for f in fields:
            f.close()


def test_batch_graph_replays(ctx):
    """Replays of the captured graph with eager work and new positions in between."""
    import torch
    import paper_1201_4060_amd as bsi
    specs = [(48, 3, 6, 30000), (32, 3, 4, 2000), (64, 3, 6, 700), (32, 3, 4, 50000)]
    fields, items = [], []
    try:
        for i, (n, C, N, P) in enumerate(specs):
            f, _ = _field(ctx, n, C, N, bsi.BSI_F32, seed=80 + i)
            fields.append(f)
            pos = dev(synth.uniform_positions(P, seed=90 + i))
            u, g = _outputs(f, P, grad=False)
            items.append((f, pos, u, g))
        with bsi.Batch(ctx, items) as b:
            for rep in range(4):
                for i, (f, pos, u, _) in enumerate(items):
                    P = pos.shape[0]
                    pos.copy_(dev(_positions(P, 1000 * rep + i, clustered=rep % 2 == 1)))
                    u.fill_(float("nan"))
                b.run(use_graph=True)
                # eager work on the same stream between replays
                junk = torch.randn(1 << 20, device="cuda").sum()
                torch.cuda.synchronize()
                for i, (f, pos, u, _) in enumerate(items):
                    us, _ = _single(f, pos, b.item_config(i), grad=False)
                    torch.cuda.synchronize()
                    assert _same(u, us), f"replay {rep} item {i}"
                log(f"  replay {rep} ok ({float(junk):.3f})")
    finally:
        for f in fields:
            f.close()


def test_batch_nonfinite_and_validation(ctx):
    import torch
    import paper_1201_4060_amd as bsi
    f1, _ = _field(ctx, 32, 3, 4, bsi.BSI_F32, seed=3)
    f2, _ = _field(ctx, 24, 3, 6, bsi.BSI_F32, seed=4)
    f3, _ = _field(ctx, 16, 3, 4, bsi.BSI_F64, seed=5)
    try:
        p = synth.uniform_positions(1000, seed=8)
        p[5] = [np.nan, 1.0, 1.0]
        p[77] = [1.0, np.inf, 2.0]
        p[900] = [1e308, 1e308, 1e308]
        pos = dev(p)
        items = [(f1, pos, *_outputs(f1, 1000)), (f2, pos, *_outputs(f2, 1000))]
        before = [f1.nonfinite_count(), f2.nonfinite_count()]
        for cfgs in ([_cfg(bsi, 8, 0), _cfg(bsi, 8, 1)], [_cfg(bsi, 4, 1), _cfg(bsi, 4, 0)]):
            with bsi.Batch(ctx, items, cfgs=cfgs) as b:
                b.run()
                torch.cuda.synchronize()
            for f, _, u, g in items:
                uh = host(u)
                bad = np.isnan(uh).any(axis=1)
                assert set(np.nonzero(bad)[0]) == {5, 77, 900}
                assert np.isnan(host(g)[[5, 77, 900]]).all()
        assert f1.nonfinite_count() - before[0] == 6 and f2.nonfinite_count() - before[1] == 6
        # one coefficient type per batch, grad for all or none, sane counts
        with pytest.raises(bsi.BsiError):
            bsi.Batch(ctx, [(f1, pos, *_outputs(f1, 1000)), (f3, pos, *_outputs(f3, 1000))])
        with pytest.raises(bsi.BsiError):
            u1, g1 = _outputs(f1, 1000)
            u2, _ = _outputs(f2, 1000)
            bsi.Batch(ctx, [(f1, pos, u1, g1), (f2, pos, u2, None)])
        with pytest.raises(bsi.BsiError):
            bsi._bsi.bsi_batch_create(ctx.handle, [])
    finally:
        for f in (f1, f2, f3):
            f.close()


def test_eval_batch_one_shot(ctx):
    import torch
    import paper_1201_4060_amd as bsi
    f1, _ = _field(ctx, 32, 3, 6, bsi.BSI_F32, seed=11)
    f2, _ = _field(ctx, 48, 1, 4, bsi.BSI_F32, seed=12)
    try:
        pa = dev(synth.uniform_positions(12345, seed=1))
        pb = dev(synth.uniform_positions(321, seed=2))
        ua, ga = _outputs(f1, 12345)
        ub, gb = _outputs(f2, 321)
        bsi._bsi.bsi_eval_batch(ctx.handle, [(f1.handle, pa, 12345, ua, ga), (f2.handle, pb, 321, ub, gb)],
                                torch.cuda.current_stream().cuda_stream)
        for f, pos, u, g in ((f1, pa, ua, ga), (f2, pb, ub, gb)):
            cfg = bsi._bsi.bsi_ctx_lookup_config(ctx.handle, f.handle, pos.shape[0])
            us, gs = f.eval(pos, cfg=cfg)
            torch.cuda.synchronize()
            log(f"  one-shot: tuned tile {cfg.sort_tile} variant {cfg.variant}")
            # the planner maps tiled sort tiles onto 4 or 8; results never depend on it
            assert _same(u, us) and _same(g, gs)
    finally:
        f1.close()
        f2.close()


def test_tuner_roundtrip(ctx, tmp_path):
    import torch
    import paper_1201_4060_amd as bsi
    f, grid = _field(ctx, 48, 3, 6, bsi.BSI_F32, seed=13)
    try:
        db = str(tmp_path / "tune.jsonl")
        best, us = bsi._bsi.bsi_tune(f.handle, 50000, seed=3, db_path=db)
        log(f"  tuned 48^3 N=6 P=5e4: tile {best.sort_tile} variant {best.variant} "
            f"tpg {best.tiles_per_group}: {us:.1f} us")
        assert us > 0
        got = bsi._bsi.bsi_ctx_lookup_config(ctx.handle, f.handle, 50000)
        assert (got.sort_tile, got.variant, got.tiles_per_group, got.tile_block, got.item_rounds) == \
            (best.sort_tile, best.variant, best.tiles_per_group, best.tile_block, best.item_rounds)
        text = open(db).read().strip().splitlines()
        assert len(text) == 1 and '"order":6' in text[0]
        with bsi.Context(0) as c2:
            bsi._bsi.bsi_ctx_load_tuning(c2.handle, db)
            with bsi.Field(c2, 48, 3, 6, bsi.BSI_F32) as f2:
                got2 = bsi._bsi.bsi_ctx_lookup_config(c2.handle, f2.handle, 50000)
                assert (got2.sort_tile, got2.variant, got2.tile_block, got2.item_rounds) == \
                    (best.sort_tile, best.variant, best.tile_block, best.item_rounds)
        # the tuned choice gives the same bits as any other configuration
        pos = dev(synth.uniform_positions(50000, seed=9))
        u0, g0 = f.eval(pos)
        u1, g1 = f.eval(pos, cfg=_cfg(bsi, 0, 1))
        torch.cuda.synchronize()
        assert _same(u0, u1) and _same(g0, g1)
        bad = tmp_path / "bad.jsonl"
        bad.write_text('{"order":5}\n')
        with pytest.raises(bsi.BsiError):
            bsi._bsi.bsi_ctx_load_tuning(ctx.handle, str(bad))
    finally:
        f.close()


def _bench_batch_specs(count=64):
    """The 64-field batching workload: field f has n uniform over
    {64,128,192,256}, order uniform over {4,6} and P = round(10^U(3,6))
    particles, drawn from stream 13 of seed 300+f (the same draws as the
    benchmark's batching form)."""
    from synth.rng import keyed_uniform
    specs = []
    for f in range(count):
        u = keyed_uniform(300 + f, 13, np.arange(3))
        n = (64, 128, 192, 256)[min(int(u[0] * 4), 3)]
        N = (4, 6)[min(int(u[1] * 2), 1)]
        specs.append((n, N, int(round(10 ** (3 + 3 * u[2])))))
    return specs


def test_batch_full_size_sampled():
    # the batching workload at its full size (64 FP32 fields, 1.3e7 particles,
    # tuned as the benchmark tunes it, graph replay): every item bitwise equal
    # to its single-field evaluation, and a sample of every item within 1e-5
    # of the oracle -- end to end (the oracle's own prefilter of the host
    # spectrum, Section 7) for every field up to 192^3 and two of the 256^3
    # ones, on the field's stored grid for the other 256^3 ones
    import torch
    import paper_1201_4060_amd as bsi
    from oracle import evaluate, prefilter
    specs = _bench_batch_specs()
    log(f"full-size batch: {len(specs)} fields, {sum(s[2] for s in specs)} particles")
    with bsi.Context(0) as c:
        fields, items, spec_buf = [], [], {}
        for f, (n, N, Pf) in enumerate(specs):
            if n not in spec_buf:
                spec_buf[n] = torch.empty((3, n, n, n // 2 + 1), dtype=torch.complex128, device="cuda")
            bsi._bsi.bsi_synth_kolmogorov(c.handle, n, 3, 300 + f, spec_buf[n])
            fld = bsi.Field(c, n, 3, N, bsi.BSI_F32)
            fld.set_spectrum(spec_buf[n])
            pos = dev(synth.uniform_positions(Pf, seed=400 + f))
            fields.append(fld)
            items.append((fld, pos) + _outputs(fld, Pf))
        del spec_buf
        tuned = set()
        for (n, N, Pf), fld in zip(specs, fields):
            key = (N, round(np.log2(Pf / n ** 3)))
            if key not in tuned:
                tuned.add(key)
                bsi._bsi.bsi_tune(fld.handle, Pf, seed=len(tuned))
        try:
            with bsi.Batch(c, items) as b:
                for _ in range(2):
                    b.run(use_graph=True)
                torch.cuda.synchronize()
                rng = np.random.default_rng(77)
                big = 0
                end_to_end = 0
                for i, ((n, N, Pf), (fld, pos, u, g)) in enumerate(zip(specs, items)):
                    su, sg = _single(fld, pos, b.item_config(i))
                    torch.cuda.synchronize()
                    assert _same(u, su) and _same(g, sg), f"item {i}"
                    pick = rng.choice(Pf, size=min(Pf, 48), replace=False)
                    if n <= 192 or big < 2:
                        big += n == 256
                        end_to_end += 1
                        grid = prefilter(synth.kolmogorov_spectrum(n, 3, seed=300 + i), N)
                    else:
                        grid = host(fld.get_coefficients())
                    wu, wg = evaluate(grid, host(pos)[pick], N)
                    eu = rel_err(host(u)[pick], wu).max()
                    eg = rel_err(host(g)[pick], wg).max()
                    assert eu < TOL_F32 and eg < TOL_F32, (i, n, N, Pf, eu, eg)
                    del grid
            log(f"  64 items bitwise equal to single-field runs and within {TOL_F32} of the oracle "
                f"({end_to_end} of them against the oracle's own prefilter)")
        finally:
            for fld in fields:
                fld.close()
