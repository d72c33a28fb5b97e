"""The comparison methods of Section 8 on the GPU: Lagrange (orders 4 and 6),
linear (order 2) and cubic Hermite, through the same evaluation kernels as the
B-spline, against the oracle (oracle.evaluate with basis="lagrange",
oracle.hermite).  Tolerances as everywhere: 1e-12 (FP64), 1e-5 (FP32 and BF16
arithmetic, the oracle on the stored coefficients), per output quantity
relative to its largest magnitude."""
import numpy as np
import pytest

import synth
from gpu_common import log, dev, host, rel_err, bf16_round, edge_positions, TOL_F64, TOL_F32

pytestmark = pytest.mark.gpu

DT = None


@pytest.fixture(scope="module")
def ctx():
    from paper_1201_4060_amd import Context
    c = Context(0)
    yield c
    c.close()


def _dt(bsi, coef):
    return {"f64": bsi.BSI_F64, "f32": bsi.BSI_F32, "bf16": bsi.BSI_BF16}[coef]


def _stored(grid, coef):
    return grid if coef == "f64" else (grid.astype(np.float32).astype(np.float64) if coef == "f32"
                                       else bf16_round(grid))


def _positions(P, seed):
    return np.concatenate([synth.uniform_positions(P, seed=seed),
                           np.random.default_rng(seed).uniform(-20, 20, size=(100, 3)), edge_positions()])


CONFIGS = (None, (8, 256, 1, 0), (8, 256, 1, 1), (0, 256, 0, 0), (4, 128, 1, 1))


def _configs(bsi):
    out = []
    for c in CONFIGS:
        out.append(None if c is None else bsi.EvalConfig(sort_tile=c[0], block=c[1], xcd_remap=c[2], variant=c[3]))
    return out


@pytest.mark.parametrize("N", [2, 4, 6])
@pytest.mark.parametrize("coef", ["f64", "f32", "bf16"])
def test_lagrange_matches_oracle(ctx, N, coef):
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate
    from oracle.symbol import NONE
    n, C = 24, 3
    uhat = synth.kolmogorov_spectrum(n, C, seed=80 + N)
    vals = prefilter(uhat, N, NONE)
    pos = _positions(4000, seed=81)
    stored = _stored(vals, coef)
    wu, wg = evaluate(stored, pos, N, basis="lagrange")
    tol = TOL_F64 if coef == "f64" else TOL_F32
    with bsi.Field(ctx, n, C, N, _dt(bsi, coef), prefilter=bsi.BSI_PREFILTER_NONE,
                   basis=bsi.BSI_BASIS_LAGRANGE) as f:
        f.set_coefficients(dev(vals))
        first = None
        for cfg in _configs(bsi):
            u, g = f.eval(dev(pos), cfg=cfg)
            u, g = host(u), host(g)
            eu, eg = rel_err(u, wu).max(), rel_err(g, wg).max()
            assert eu < tol and eg < tol, (cfg, eu, eg)
            if first is None:
                first = (u, g)
                log(f"  lagrange N={N} {coef}: max rel err u {eu:.2e} grad {eg:.2e}")
            else:   # every gather variant runs the same arithmetic
                assert np.array_equal(u, first[0], equal_nan=True) and np.array_equal(g, first[1], equal_nan=True)


@pytest.mark.parametrize("N", [2, 4, 6])
def test_lagrange_end_to_end_from_spectrum(ctx, N):
    # the GPU's inverse FFT with c = 1 gives the grid values; the interpolant
    # passes through them (interpolation property) and matches the oracle
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate
    from oracle.symbol import NONE
    n, C = 32, 3
    uhat = synth.kolmogorov_spectrum(n, C, seed=85)
    vals = prefilter(uhat, N, NONE)
    pos = _positions(3000, seed=86)
    wu, wg = evaluate(vals, pos, N, basis="lagrange")
    for coef, tol in (("f64", TOL_F64), ("f32", TOL_F32)):
        with bsi.Field(ctx, n, C, N, _dt(bsi, coef), prefilter=bsi.BSI_PREFILTER_NONE,
                       basis=bsi.BSI_BASIS_LAGRANGE) as f:
            f.set_spectrum(dev(uhat))
            grid = host(f.get_coefficients())
            assert np.max(np.abs(grid - vals)) < (1e-12 if coef == "f64" else 1e-6) * np.abs(vals).max()
            u, g = f.eval(dev(pos))
            eu, eg = rel_err(host(u), wu).max(), rel_err(host(g), wg).max()
            log(f"  lagrange N={N} {coef} from the spectrum: max rel err u {eu:.2e} grad {eg:.2e}")
            assert eu < tol and eg < tol
            nodes = np.random.default_rng(87).integers(0, n, size=(500, 3))
            un, _ = f.eval(dev(nodes * (2 * np.pi / n)))
            want = vals[:, nodes[:, 0], nodes[:, 1], nodes[:, 2]].T
            assert np.max(np.abs(host(un) - want)) < (1e-13 if coef == "f64" else 1e-6) * np.abs(vals).max()


def test_linear_bspline_equals_linear_lagrange(ctx):
    # order 2: the B-spline matrix M_(2) is linear interpolation, and with
    # prefilter NONE the two fields give bitwise equal results; with the
    # L2-optimal c the order-2 B-spline matches the oracle
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate
    n, C = 32, 3
    uhat = synth.kolmogorov_spectrum(n, C, seed=88)
    pos = dev(_positions(3000, seed=89))
    with bsi.Field(ctx, n, C, 2, bsi.BSI_F64, prefilter=bsi.BSI_PREFILTER_NONE) as fb, \
            bsi.Field(ctx, n, C, 2, bsi.BSI_F64, prefilter=bsi.BSI_PREFILTER_NONE,
                      basis=bsi.BSI_BASIS_LAGRANGE) as fl, \
            bsi.Field(ctx, n, C, 2, bsi.BSI_F64) as fo:
        spec = dev(uhat)
        for f in (fb, fl, fo):
            f.set_spectrum(spec)
        ub, gb = fb.eval(pos)
        ul, gl = fl.eval(pos)
        assert np.array_equal(host(ub), host(ul), equal_nan=True)
        assert np.array_equal(host(gb), host(gl), equal_nan=True)
        uo, go = fo.eval(pos)
        wu, wg = evaluate(prefilter(uhat, 2), host(pos), 2)
        assert rel_err(host(uo), wu).max() < TOL_F64 and rel_err(host(go), wg).max() < TOL_F64


@pytest.mark.parametrize("coef", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("C", [1, 3])
def test_hermite_matches_oracle(ctx, coef, C):
    import paper_1201_4060_amd as bsi
    from oracle import hermite
    n = 24
    uhat = synth.kolmogorov_spectrum(n, C, seed=90 + C)
    dg = hermite.derivative_grids(uhat)
    inter = hermite.interleaved(dg)
    stored = _stored(inter, coef)
    sd = {a: stored[:, a[0]::2, a[1]::2, a[2]::2] for a in hermite.ORDERS}
    pos = _positions(4000, seed=91)
    wu, wg = hermite.evaluate_hermite(sd, pos)
    tol = TOL_F64 if coef == "f64" else TOL_F32
    with bsi.Field(ctx, n, C, 4, _dt(bsi, coef), prefilter=bsi.BSI_PREFILTER_NONE,
                   basis=bsi.BSI_BASIS_HERMITE) as f:
        f.set_coefficients(dev(inter))
        assert np.array_equal(host(f.get_coefficients()), stored)
        first = None
        for cfg in _configs(bsi):
            u, g = f.eval(dev(pos), cfg=cfg)
            u, g = host(u), host(g)
            eu, eg = rel_err(u, wu).max(), rel_err(g, wg).max()
            assert eu < tol and eg < tol, (cfg, eu, eg)
            if first is None:
                first = (u, g)
                log(f"  hermite C={C} {coef}: max rel err u {eu:.2e} grad {eg:.2e}")
            else:
                assert np.array_equal(u, first[0], equal_nan=True) and np.array_equal(g, first[1], equal_nan=True)


@pytest.mark.parametrize("n", [32, 48])
def test_hermite_end_to_end_from_spectrum(ctx, n):
    # 8 inverse FFTs on the GPU (one per derivative field, Table 2) against the
    # oracle's spectral derivatives, then the interpolant
    import paper_1201_4060_amd as bsi
    from oracle import hermite
    C = 3
    uhat = synth.kolmogorov_spectrum(n, C, seed=93)
    dg = hermite.derivative_grids(uhat)
    inter = hermite.interleaved(dg)
    pos = _positions(3000, seed=94)
    wu, wg = hermite.evaluate_hermite(dg, pos)
    for coef, tol in (("f64", TOL_F64), ("f32", TOL_F32)):
        with bsi.Field(ctx, n, C, 4, _dt(bsi, coef), prefilter=bsi.BSI_PREFILTER_NONE,
                       basis=bsi.BSI_BASIS_HERMITE) as f:
            f.set_spectrum(dev(uhat))
            grid = host(f.get_coefficients())
            for a in hermite.ORDERS:
                part = grid[:, a[0]::2, a[1]::2, a[2]::2]
                d = np.max(np.abs(part - dg[a])) / np.abs(dg[a]).max()
                assert d < (1e-12 if coef == "f64" else 1e-5), (coef, a, d)
            u, g = f.eval(dev(pos))
            eu, eg = rel_err(host(u), wu).max(), rel_err(host(g), wg).max()
            log(f"  hermite n={n} {coef} from the spectrum: max rel err u {eu:.2e} grad {eg:.2e}")
            assert eu < tol and eg < tol


def test_methods_full_size_sampled(ctx):
    # 128^3 x3 FP32: Lagrange order 4 and Hermite end to end, 10^6 particles,
    # a sample against the oracle
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate, hermite
    from oracle.symbol import NONE
    n, C = 128, 3
    uhat = synth.kolmogorov_spectrum(n, C, seed=95)
    pos = synth.uniform_positions(1_000_000, seed=96)
    pick = np.sort(np.random.default_rng(97).choice(pos.shape[0], 2000, replace=False))
    spec = dev(uhat)
    with bsi.Field(ctx, n, C, 4, bsi.BSI_F32, prefilter=bsi.BSI_PREFILTER_NONE,
                   basis=bsi.BSI_BASIS_LAGRANGE) as fl, \
            bsi.Field(ctx, n, C, 4, bsi.BSI_F32, prefilter=bsi.BSI_PREFILTER_NONE,
                      basis=bsi.BSI_BASIS_HERMITE) as fh:
        fl.set_spectrum(spec)
        fh.set_spectrum(spec)
        ul, gl = fl.eval(dev(pos))
        uh, gh = fh.eval(dev(pos))
        ul, gl, uh, gh = host(ul)[pick], host(gl)[pick], host(uh)[pick], host(gh)[pick]
    wu, wg = evaluate(prefilter(uhat, 4, NONE), pos[pick], 4, basis="lagrange")
    assert rel_err(ul, wu).max() < TOL_F32 and rel_err(gl, wg).max() < TOL_F32
    hu, hg = hermite.evaluate_hermite(hermite.derivative_grids(uhat), pos[pick])
    eu, eg = rel_err(uh, hu).max(), rel_err(gh, hg).max()
    log(f"  128^3 hermite sampled: max rel err u {eu:.2e} grad {eg:.2e}")
    assert eu < TOL_F32 and eg < TOL_F32


def test_method_validation(ctx):
    import torch
    import paper_1201_4060_amd as bsi
    from paper_1201_4060_amd import _bsi
    with pytest.raises(bsi.BsiError) as e:    # Lagrange needs the grid values
        bsi.Field(ctx, 16, 1, 4, bsi.BSI_F32, basis=bsi.BSI_BASIS_LAGRANGE)
    assert e.value.status == 1
    with pytest.raises(bsi.BsiError) as e:
        bsi.Field(ctx, 16, 1, 6, bsi.BSI_F32, prefilter=bsi.BSI_PREFILTER_NONE, basis=bsi.BSI_BASIS_HERMITE)
    assert e.value.status == 3
    with pytest.raises(bsi.BsiError) as e:
        bsi.Field(ctx, 16, 1, 4, bsi.BSI_F32, basis=7)
    assert e.value.status == 1
    with bsi.Field(ctx, 16, 3, 4, bsi.BSI_F32, prefilter=bsi.BSI_PREFILTER_NONE,
                   basis=bsi.BSI_BASIS_LAGRANGE) as f:
        pos = dev(synth.uniform_positions(10, seed=1))
        with pytest.raises(bsi.BsiError) as e:
            f.eval_hessian(pos)
        assert e.value.status == 3
        u = torch.empty((10, 3), dtype=torch.float32, device="cuda")
        with pytest.raises(bsi.BsiError) as e:
            bsi.Batch(ctx, [(f, pos, u, None)])
        assert e.value.status == 3
