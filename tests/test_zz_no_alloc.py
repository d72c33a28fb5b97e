"""The allocation-free evaluation entry point (bsi_eval_static) against the
regular one (bsi_eval_ex) with the same configuration: bitwise equal outputs,
two calls in a row (the second smaller), no device allocation by the call,
and a clear error beyond the static workspace."""
import numpy as np
import pytest

import synth
from gpu_common import log, dev, host

pytestmark = pytest.mark.gpu


def _free_bytes():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_static_matches_regular_twice():
    import torch
    import paper_1201_4060_amd as bsi
    from paper_1201_4060_amd import _bsi
    n, C, N = 64, 3, 6
    with bsi.Context(0) as ctx, bsi.Field(ctx, n, C, N, bsi.BSI_F32) as f:
        f.set_spectrum(dev(synth.kolmogorov_spectrum(n, C, seed=90)))
        cfgs = [None, bsi.EvalConfig(sort_tile=8, block=256, xcd_remap=1),
                bsi.EvalConfig(sort_tile=4, block=128, variant=1), bsi.EvalConfig(sort_tile=0, block=256)]
        # one untimed round first: the HIP runtime sets up per-process launch
        # resources of its own on the first launches of the library's kernels
        warm = dev(synth.uniform_positions(1000, seed=89))
        wu = torch.empty((1000, C), dtype=torch.float32, device="cuda")
        wg = torch.empty((1000, C, 3), dtype=torch.float32, device="cuda")
        for cfg in cfgs:
            _bsi.bsi_eval_static(f.handle, warm, 1000, wu, wg, cfg)
        torch.cuda.synchronize()
        for P in (400_000, 37_001):              # the second call is smaller
            pos = dev(np.concatenate([synth.clustered_positions(P // 2, 4, P // 8, 0.2, seed=91 + P)[:P - 2],
                                      [[np.nan, 1.0, 1.0], [np.inf, 2.0, 3.0]]]))
            for cfg in cfgs:
                u0 = torch.full((P, C), float("nan"), dtype=torch.float32, device="cuda")
                g0 = torch.full((P, C, 3), float("nan"), dtype=torch.float32, device="cuda")
                u1, g1 = torch.zeros_like(u0), torch.zeros_like(g0)
                free0 = _free_bytes()
                _bsi.bsi_eval_static(f.handle, pos, P, u0, g0, cfg)
                free1 = _free_bytes()
                _bsi.bsi_eval_ex(f.handle, pos, P, u1, g1, cfg)
                torch.cuda.synchronize()
                log(f"  P={P} cfg={None if cfg is None else (cfg.sort_tile, cfg.variant)}: "
                    f"free memory change {free0 - free1} bytes")
                assert free0 - free1 < (1 << 20), "the static entry point allocated device memory"
                assert np.array_equal(host(u0), host(u1), equal_nan=True)
                assert np.array_equal(host(g0), host(g1), equal_nan=True)
                assert np.isnan(host(u0)[-2:]).all() and np.isfinite(host(u0)[:-2]).all()
        # value only, and a call on the context's own stream
        P = 5000
        pos = dev(synth.uniform_positions(P, seed=93))
        u0 = torch.empty((P, C), dtype=torch.float32, device="cuda")
        u1 = torch.empty_like(u0)
        _bsi.bsi_eval_static(f.handle, pos, P, u0, None, None)
        _bsi.bsi_eval_ex(f.handle, pos, P, u1, None, None)
        torch.cuda.synchronize()
        assert np.array_equal(host(u0), host(u1))


def test_static_rejects_oversized_workspace():
    import torch
    import paper_1201_4060_amd as bsi
    from paper_1201_4060_amd import _bsi
    with bsi.Context(0) as ctx, bsi.Field(ctx, 32, 1, 4, bsi.BSI_F64) as f:
        P = 4_000_000                            # about 280 MB of binning workspace
        pos = torch.zeros((P, 3), dtype=torch.float64, device="cuda")
        u = torch.empty((P, 1), dtype=torch.float64, device="cuda")
        cfg = bsi.EvalConfig(sort_tile=8, block=256)
        with pytest.raises(bsi.BsiError) as e:
            _bsi.bsi_eval_static(f.handle, pos, P, u, None, cfg)
        assert e.value.status == 1 and "static maximum" in str(e.value)
        log(f"  {e.value}")
        # an unbinned configuration needs no workspace at any size
        _bsi.bsi_eval_static(f.handle, pos[:1000], 1000, u, None, bsi.EvalConfig(sort_tile=0, block=256))
        torch.cuda.synchronize()
