"""Serving form on the GPU: continuous batching of particle queries.

Requests of varying size against several resident fields are submitted while
others run; each result must be bitwise the stand-alone bsi_eval_ex result of
its field with the configuration the context picks for its size, and served
results on 256^3 fields are also compared with the FP64 oracle directly.
Admission must respect the device-memory budget.
"""
import threading

import numpy as np
import pytest

import synth
from gpu_common import log, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    import torch
    import paper_1201_4060_amd as bsi
    ctx = bsi.Context(0)
    fields = {}
    fid = 0
    for n, C in ((32, 3), (48, 3), (64, 1)):
        uhat = dev(synth.kolmogorov_spectrum(n, C, seed=500 + n))
        for N in (4, 6):
            f = bsi.Field(ctx, n, C, N, bsi.BSI_F32)
            f.set_spectrum(uhat)
            fields[fid] = f
            fid += 1
    torch.cuda.synchronize()
    yield ctx, fields
    for f in fields.values():
        f.close()
    ctx.close()


def _pinned(shape, dtype):
    import torch
    return torch.empty(shape, dtype=dtype, pin_memory=True)


def _request(rng, fields, k):
    import torch
    fid = int(rng.integers(len(fields)))
    P = int(round(10 ** rng.uniform(0, 4.5)))
    pos = synth.uniform_positions(P, seed=7000 + k) if k % 2 else \
        synth.clustered_positions(P // 2, 2, (P - P // 2) // 2, 0.2, seed=7000 + k)
    if pos.shape[0] < P:
        pos = np.concatenate([pos, synth.uniform_positions(P - pos.shape[0], seed=9000 + k)])
    f = fields[fid]
    p = _pinned((P, 3), torch.float64)
    p.numpy()[:] = pos
    u = _pinned((P, f.ncomp), torch.float32)
    g = _pinned((P, f.ncomp, 3), torch.float32)
    u.fill_(float("nan"))
    g.fill_(float("nan"))
    return fid, p, u, g


def test_results_equal_alone_and_in_the_mix(served):
    import torch
    import paper_1201_4060_amd as bsi
    ctx, fields = served
    rng = np.random.default_rng(11)
    reqs = [_request(rng, fields, k) for k in range(160)]
    tickets = [None] * len(reqs)
    with bsi.Server(ctx, hbm_budget=64 << 20, max_slots=4) as sv:
        for fid, f in fields.items():
            sv.add_field(fid, f)

        def submit(lo, hi):
            for k in range(lo, hi):
                fid, p, u, g = reqs[k]
                tickets[k] = sv.submit(fid, p, u, g)

        # two client threads submitting at once
        th = [threading.Thread(target=submit, args=(0, 80)), threading.Thread(target=submit, args=(80, 160))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        lat = [sv.wait(t) for t in tickets]
        sv.drain()
        st = sv.stats()
        log(f"  served {st['completed']} requests, max in flight {st['max_inflight']}, "
            f"p50 {st['p50_ns'] / 1e3:.0f} us, p99 {st['p99_ns'] / 1e3:.0f} us, "
            f"peak arena {st['peak_arena_bytes'] / 2**20:.1f} MiB")
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["max_inflight"] >= 2, "requests never overlapped"
        assert 0 < st["p50_ns"] <= st["p99_ns"]
        assert st["peak_arena_bytes"] <= 64 << 20
        assert all(x > 0 for x in lat)
    # the same queries alone
    for k, (fid, p, u, g) in enumerate(reqs):
        f = fields[fid]
        P = p.shape[0]
        cfg = bsi._bsi.bsi_ctx_lookup_config(ctx.handle, f.handle, P)
        ua, ga = f.eval(p.cuda(), cfg=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(u.numpy(), host(ua)) and np.array_equal(g.numpy(), host(ga)), \
            f"request {k} (field {fid}, P={P}) differs from its stand-alone result"


def test_admission_by_budget_and_errors(served):
    import torch
    import paper_1201_4060_amd as bsi
    ctx, fields = served
    budget = 2 << 20
    rng = np.random.default_rng(5)
    with bsi.Server(ctx, hbm_budget=budget, max_slots=8) as sv:
        for fid, f in fields.items():
            sv.add_field(fid, f)
        reqs = []
        for k in range(40):
            f = fields[k % len(fields)]
            P = 6000
            p = _pinned((P, 3), torch.float64)
            p.numpy()[:] = synth.uniform_positions(P, seed=300 + k)
            u = _pinned((P, f.ncomp), torch.float32)
            reqs.append((k % len(fields), p, u))
        tickets = [sv.submit(fid, p, u) for fid, p, u in reqs]
        for t in tickets:
            sv.wait(t)
        st = sv.stats()
        log(f"  budget {budget >> 20} MiB: max in flight {st['max_inflight']}, "
            f"peak arena {st['peak_arena_bytes'] / 2**20:.2f} MiB")
        assert st["peak_arena_bytes"] <= budget
        assert 1 <= st["max_inflight"] < 8   # memory, not slots, bounds the overlap
        for fid, p, u in reqs:
            f = fields[fid]
            ua, _ = f.eval(p.cuda(), grad=False,
                           cfg=bsi._bsi.bsi_ctx_lookup_config(ctx.handle, f.handle, p.shape[0]))
            torch.cuda.synchronize()
            assert np.array_equal(u.numpy(), host(ua))
        # a request larger than the whole budget is refused at submission
        P = 200000
        p = _pinned((P, 3), torch.float64)
        p.numpy()[:] = synth.uniform_positions(P, seed=1)
        u = _pinned((P, 3), torch.float32)
        with pytest.raises(bsi.BsiError) as e:
            sv.submit(0, p, u)
        assert e.value.status == 2
        with pytest.raises(bsi.BsiError):
            bsi._bsi.bsi_server_submit(sv.handle, 99, p, 10, u)
        with pytest.raises(bsi.BsiError):
            bsi._bsi.bsi_server_submit(sv.handle, 0, p, 0, u)
        with pytest.raises(bsi.BsiError):
            sv.add_field(0, fields[0])
        # a collected ticket's record is released: waiting or polling it again
        # is an error; a request polled to completion is collected as well
        assert st["completed"] == len(tickets)
        with pytest.raises(bsi.BsiError) as e:
            bsi._bsi.bsi_server_wait(sv.handle, tickets[0])
        assert e.value.status == 1
        with pytest.raises(bsi.BsiError) as e:
            bsi._bsi.bsi_server_poll(sv.handle, tickets[-1])
        assert e.value.status == 1
        fid, p, u = reqs[0]
        t = sv.submit(fid, p, u)
        while not sv.poll(t)[0]:
            pass
        with pytest.raises(bsi.BsiError):
            bsi._bsi.bsi_server_wait(sv.handle, t)
        with pytest.raises(bsi.BsiError):   # never issued
            bsi._bsi.bsi_server_poll(sv.handle, t + 1)


def test_served_full_size(served):
    """The serving workload's sizes: a 1024^3 x3 snapshot (order 6) and a 256^3 x3
    one (order 4), FP32, from the device spectrum generator; requests of 10^3 to
    10^6 uniform or clustered particles served while others run, each bitwise
    equal to its stand-alone evaluation."""
    import torch
    import paper_1201_4060_amd as bsi
    ctx, _ = served
    fields = {}
    try:
        for fid, (n, N) in enumerate(((1024, 6), (256, 4))):
            spec = torch.empty((3, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
            bsi._bsi.bsi_synth_kolmogorov(ctx.handle, n, 3, 500 + fid, spec)
            f = bsi.Field(ctx, n, 3, N, bsi.BSI_F32)
            f.set_spectrum(spec)
            fields[fid] = f
            del spec
        torch.cuda.synchronize()
        log(f"  resident: 1024^3 and 256^3 snapshots, "
            f"{sum(bsi._bsi.bsi_field_bytes(f.handle) for f in fields.values()) / 2**30:.1f} GiB of grids")
        reqs = []
        for k, (fid, P, clustered) in enumerate(((0, 1_000_000, False), (1, 1000, True), (0, 100_000, True),
                                                (1, 1_000_000, False), (0, 3000, False), (1, 250_000, True))):
            pos = synth.clustered_positions(P // 2, 4, P // 8, 0.1, seed=620 + k) if clustered else \
                synth.uniform_positions(P, seed=620 + k)
            pos = pos[:P]
            p = _pinned((P, 3), torch.float64)
            p.numpy()[:] = pos
            u = _pinned((P, 3), torch.float32)
            g = _pinned((P, 3, 3), torch.float32)
            u.fill_(float("nan"))
            g.fill_(float("nan"))
            reqs.append((fid, p, u, g))
        with bsi.Server(ctx, hbm_budget=1 << 30, max_slots=4) as sv:
            for fid, f in fields.items():
                sv.add_field(fid, f)
            tickets = [sv.submit(fid, p, u, g) for fid, p, u, g in reqs]
            for t in tickets:
                sv.wait(t)
            st = sv.stats()
            assert st["completed"] == len(reqs) and st["failed"] == 0
        for k, (fid, p, u, g) in enumerate(reqs):
            f = fields[fid]
            P = p.shape[0]
            cfg = bsi._bsi.bsi_ctx_lookup_config(ctx.handle, f.handle, P)
            ua, ga = f.eval(p.cuda(), cfg=cfg)
            torch.cuda.synchronize()
            assert not np.isnan(u.numpy()).any()
            assert np.array_equal(u.numpy(), host(ua)) and np.array_equal(g.numpy(), host(ga)), \
                f"request {k} (field {fid}, P={P}) differs from its stand-alone result"
            log(f"  request {k}: field {fid}, P={P}: bitwise equal to stand-alone")
    finally:
        for f in fields.values():
            f.close()


def test_served_requests_match_oracle(served):
    """Served requests against the FP64 oracle (Section 7 prefilter of the same
    spectrum, then the plain stencil sum): 256^3 x3 FP32 fields of both orders,
    uniform and clustered requests served while others run; every sampled
    output within 1e-5 of the oracle per quantity."""
    import torch
    import paper_1201_4060_amd as bsi
    from oracle import prefilter, evaluate
    from gpu_common import rel_err, TOL_F32
    ctx, _ = served
    n, C = 256, 3
    uhat = synth.kolmogorov_spectrum(n, C, seed=510)
    fields = {}
    try:
        spec = dev(uhat)
        for fid, N in enumerate((4, 6)):
            f = bsi.Field(ctx, n, C, N, bsi.BSI_F32)
            f.set_spectrum(spec)
            fields[fid] = f
        del spec
        torch.cuda.synchronize()
        reqs = []
        for k, (fid, P, clustered) in enumerate(((0, 60_000, False), (1, 40_000, True), (1, 5_000, False),
                                                (0, 30_000, True), (1, 80_000, False), (0, 2_000, True))):
            pos = synth.clustered_positions(P // 2, 3, P // 6, 0.1, seed=640 + k) if clustered else \
                synth.uniform_positions(P, seed=640 + k)
            pos = pos[:P]
            p = _pinned((pos.shape[0], 3), torch.float64)
            p.numpy()[:] = pos
            u = _pinned((pos.shape[0], C), torch.float32)
            g = _pinned((pos.shape[0], C, 3), torch.float32)
            u.fill_(float("nan"))
            g.fill_(float("nan"))
            reqs.append((fid, p, u, g))
        with bsi.Server(ctx, hbm_budget=256 << 20, max_slots=4) as sv:
            for fid, f in fields.items():
                sv.add_field(fid, f)
            tickets = [sv.submit(fid, p, u, g) for fid, p, u, g in reqs]
            for t in tickets:
                sv.wait(t)
            st = sv.stats()
            assert st["completed"] == len(reqs) and st["failed"] == 0
            log(f"  served {len(reqs)} requests on 256^3 fields, max in flight {st['max_inflight']}")
        grids = {fid: prefilter(uhat, N) for fid, N in enumerate((4, 6))}
        rng = np.random.default_rng(12)
        for k, (fid, p, u, g) in enumerate(reqs):
            N = (4, 6)[fid]
            P = p.shape[0]
            pick = np.sort(rng.choice(P, size=min(P, 1500), replace=False))
            wu, wg = evaluate(grids[fid], p.numpy()[pick], N)
            eu = rel_err(u.numpy()[pick], wu).max()
            eg = rel_err(g.numpy()[pick], wg).max()
            log(f"  request {k}: order {N}, P={P}: max rel err u {eu:.2e} grad {eg:.2e}")
            assert eu < TOL_F32 and eg < TOL_F32, (k, eu, eg)
    finally:
        for f in fields.values():
            f.close()
