#!/usr/bin/env python3
"""Throughput benchmark of the B-spline interpolation hot path on one MI355X.

Default workload (--form precision): a 512^3 three-component divergence-free
Kolmogorov field (spectrum |uhat|^2 ~ k^-11/3, cut-off |k| <= n/3, complex128
input), spline order 6, 10^7 clustered particles (half uniform, half in 100
Gaussian blobs, sigma 0.1).  One step runs the whole path on the FP32
coefficient grid: prefilter (FP64 symbol multiply + inverse 3D real FFT), then
evaluation (cell/Morton binning + gather) of u and grad u at every particle.
value = particles per second of whole step, inputs resident in HBM.  The same
step on the BF16 grid and on the plain FP64 grid is timed on the same inputs
(legs), every path's error against the FP64 oracle is reported, and the serving
form's latency percentiles are attached.

Other forms (one JSON line each, same keys):
  --form plain      256^3 x3 field, FP32 grid, orders 4 and 6, 10^6 uniform
                    particles; step = prefilter + eval per order
  --form batch      64 fields (n in {64,128,192,256}, order 4|6, 10^3..10^6
                    particles each) in one persistent gather launch replayed
                    from a HIP graph; beside it one launch per field
  --form serve      resident 1024^3 and 256^3 fields (both orders), Poisson
                    particle-query requests; points/s with p50/p99 latency
  --form hessian    the plain workload with second derivatives as well
  --form copy       1 GiB device copy (calibrates HBM byte counters)

Prints one JSON line on stdout; diagnostics go to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "interp points/s (u+∇u), HBM GB/s vs peak; p99 latency at fixed request rate"
HBM_PEAK_GBS = 8000.0
N_GRID = 256
NCOMP = 3
ORDERS = (4, 6)
P = 1_000_000
FIELD_SEED, POS_SEED = 1, 101
STAGES = ("fft_axis0", "fft_axis1", "fft_c2r", "bin_count", "bin_scan", "bin_scatter", "bin_items", "gather")
EVAL_STAGES = ("bin_count", "bin_scan", "bin_scatter", "bin_items", "gather")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_256cube_x3_f32_orders4_6_1e6.md")
KERNEL_SOURCES = {"gather": ["eval.hip", "gather.hpp", "common.hpp"], "fft": ["fft.hip", "common.hpp"]}


def eprint(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------ byte counts ---

def distinct_stencil_points(pos, n, order, mark=None):
    """Number of distinct grid points in the union of all particles' stencils.

    pos: torch float64 device tensor [P][3] on [0, 2pi)^3 (or numpy array).
    Counted on the device with a mark array of n^3 booleans.
    """
    import torch
    if isinstance(pos, np.ndarray):
        pos = torch.from_numpy(pos).cuda()
    cell = torch.remainder(torch.floor(pos * (n / (2.0 * np.pi))).to(torch.int64), n)
    if mark is None or mark.numel() != n ** 3:
        mark = torch.zeros(n ** 3, dtype=torch.bool, device=pos.device)
    else:
        mark.zero_()
    offs = [o - order // 2 + 1 for o in range(order)]
    for a in offs:
        i0 = torch.remainder(cell[:, 0] + a, n) * (n * n)
        for b in offs:
            i01 = i0 + torch.remainder(cell[:, 1] + b, n) * n
            for e in offs:
                mark[i01 + torch.remainder(cell[:, 2] + e, n)] = True
    return int(mark.sum().item())


def gather_bytes(P_, C, U, coef_bytes, out_bytes=4):
    """Algorithmic bytes of one gather: positions (24 B) and u, grad u per
    particle, plus every distinct coefficient touched once."""
    return P_ * (24 + 4 * C * out_bytes) + U * C * coef_bytes


# FP32 FMA rate of the vector ALUs without packed FP32 (256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz); the library is compiled without packed FP32 instructions
FMA_PEAK_PER_S = 256 * 4 * 16 * 2.4e9


def gather_fma(N, C):
    """FMAs per particle of the u + grad u contraction (leading term 6N^3 for C = 3)."""
    return 6 * N ** 3 + 15 * N ** 2 + 12 * N if C == 3 else 2 * N ** 3 + 9 * N ** 2 + 4 * N


def hessian_fma(N, C):
    """FMAs per particle of the u + grad u + second-derivative contraction:
    3 per coefficient along axis 2, 6 per row along axis 1, 10 per plane."""
    return 3 * C * N ** 3 + 6 * C * N ** 2 + 10 * C * N


def fft_bytes(stage, n, C, order, spec_bytes=16, work_bytes=8, grid_bytes=4):
    """Algorithmic bytes of one FFT pass (spectrum read, work array, grid written)."""
    half = n * n * (n // 2 + 1) * C
    if stage == "fft_axis0":
        return half * (spec_bytes + work_bytes)
    if stage == "fft_axis1":
        return half * 2 * work_bytes
    if stage == "fft_c2r":
        return half * work_bytes + (n + order - 1) ** 3 * C * grid_bytes
    return None


def measured_traffic(key, path=None):
    """HBM bytes per launch of stage `key` from a committed counter summary.

    The summary records FETCH_SIZE + WRITE_SIZE (scaled by a plain copy of
    known size) with a hash of the kernel's sources; the figure is returned
    only while the sources still hash the same, else None.
    """
    try:
        text = open(path or TRAFFIC_FILE).read()
    except OSError:
        return None
    line = next((ln for ln in text.splitlines() if ln.startswith("traffic-json:")), None)
    if line is None:
        return None
    table = json.loads(line.split(":", 1)[1])
    ent = table.get(key) or table.get(key.split("@")[0])
    if ent is None:
        return None
    kind = "gather" if key.startswith("gather") else "fft"
    return ent["traffic_bytes"] if kernel_source_hash(kind) == ent["src"] else None


def kernel_source_hash(kind):
    """Hash of the kernel sources of `kind` with comments and blank space
    removed (editing a comment does not change the kernel)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1201_4060_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def roofline_entry(key, alg, avg_us, traffic=None):
    achieved = alg / (avg_us * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": key,
            "algorithmic_bytes": int(alg), "avg_us": round(avg_us, 2)}


# ---------------------------------------------------------------- timing ---

def read_stages(bsi, ctx, suffix, names=STAGES):
    out = {}
    for st in names:
        ms, cnt = bsi._bsi.bsi_ctx_read_timing(ctx.handle, st)
        if cnt:
            out[f"{st}@{suffix}"] = {"avg_us": 1000.0 * ms / cnt, "launches": cnt, "total_ms": ms}
    return out


STEP_PERCENTILES = {}  # ms per step of the last timed run (p10, p50, p90)


def timed_steps(step, warmup, steps, ctxs, bsi, stage_timing=True):
    """Run warm-up steps, then time `steps` steps (synchronised on both sides),
    with the library's per-stage kernel timing on every context if
    `stage_timing` (its events cost several % of a step: the figure a line
    reports comes from a run without them); returns seconds/step."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    for c in ctxs:
        bsi._bsi.bsi_ctx_reset_timing(c.handle)
        bsi._bsi.bsi_ctx_set_timing(c.handle, stage_timing)
    torch.cuda.synchronize()
    # an event after every step on torch's stream (the library works on it):
    # per-step durations for the percentiles, the wall clock for the mean
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    STEP_PERCENTILES.update({"p10": round(float(np.percentile(per, 10)), 4),
                             "p50": round(float(np.percentile(per, 50)), 4),
                             "p90": round(float(np.percentile(per, 90)), 4)})
    return (t1 - t0) / steps


def overlapped(parts, sides):
    """Run the independent parts of a step concurrently: parts[0] on torch's
    current stream, parts[i] on sides[i - 1] (default priority), all joined
    back into the current stream at the end."""
    import torch
    main = torch.cuda.current_stream()
    for s in sides:
        s.wait_stream(main)
    for part, s in zip(parts[1:], sides):
        with torch.cuda.stream(s):
            part()
    parts[0]()
    for s in sides:
        main.wait_stream(s)


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """GB/s (bytes read + written) of a plain 1 GiB device-to-device copy: the
    practical yardstick beside the 8 TB/s datasheet peak."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    return 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def base_line(args, value, unit, sec_per_step, dtype, config, roofline, cpu, **extra):
    line = {"metric": METRIC, "value": round(value, 1), "unit": unit, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec_per_step * 1e3, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config, "roofline": roofline}
    if STEP_PERCENTILES:
        line["ms_per_step_percentiles"] = dict(STEP_PERCENTILES)
    line.update(extra)
    line["cpu_baseline"] = cpu
    return line


def print_stages(stages, sec_per_step, steps):
    tot = sum(v["total_ms"] for v in stages.values()) / steps
    eprint(f"{sec_per_step * 1e3:.3f} ms/step wall, {tot:.3f} ms/step in library kernels")
    for k, v in sorted(stages.items(), key=lambda kv: -kv[1]["total_ms"]):
        eprint(f"  {k:22s} {v['avg_us']:9.1f} us x {v['launches']}")


# ------------------------------------------------------------ plain form ---

def cpu_baseline_plain(uhat, pos, sample):
    """Time the FP64 oracle (as it stands) on a bounded sample of the workload."""
    from threadpoolctl import threadpool_limits
    import oracle
    idx = np.random.default_rng(0).choice(pos.shape[0], sample, replace=False)
    sub = pos[idx]
    total = 0.0
    with threadpool_limits(limits=1):
        for order in ORDERS:
            t0 = time.perf_counter()
            grid = oracle.prefilter(uhat, order)
            t1 = time.perf_counter()
            oracle.evaluate(grid, sub, order)
            t2 = time.perf_counter()
            del grid
            total += (t1 - t0) + (t2 - t1) * (P / sample)
            eprint(f"cpu oracle order {order}: prefilter {t1 - t0:.2f} s, "
                   f"eval {sample} particles {t2 - t1:.2f} s")
    return {"value": len(ORDERS) * P / total, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": (f"full FP64 prefilter of the 256^3x3 field per order + evaluation of "
                       f"{sample} of the 1e6 particles per order, scaled to 1e6; numpy, one thread")}


def form_plain(args):
    import torch
    import synth
    import paper_1201_4060_amd as bsi
    dev = torch.device("cuda:0")
    eprint("generating inputs ...")
    uhat_np = synth.kolmogorov_spectrum(N_GRID, NCOMP, seed=FIELD_SEED)
    pos_np = synth.uniform_positions(P, seed=POS_SEED)
    uhat = torch.from_numpy(uhat_np).to(dev)
    pos = torch.from_numpy(pos_np).to(dev)

    ctxs = {o: bsi.Context(0) for o in ORDERS}          # one context per order: per-order stage timing
    fields = {o: bsi.Field(ctxs[o], N_GRID, NCOMP, o, bsi.BSI_F32) for o in ORDERS}
    outs = {o: (torch.empty((P, NCOMP), dtype=torch.float32, device=dev),
                torch.empty((P, NCOMP, 3), dtype=torch.float32, device=dev)) for o in ORDERS}
    cfg = None
    if args.sort_tile is not None:
        cfg = bsi.EvalConfig(sort_tile=args.sort_tile, block=256, xcd_remap=1)

    def order_part(o):
        def run():
            fields[o].set_spectrum(uhat)
            fields[o].eval(pos, cfg=cfg, out=outs[o])
        return run

    def step_one_stream():
        for o in ORDERS:
            order_part(o)()

    # the two orders are independent: with --streams 2 they run on two streams,
    # so that one order's memory-bound FFT passes overlap the other's gather
    sides = [torch.cuda.Stream() for _ in ORDERS[1:]]
    parts = [order_part(o) for o in ORDERS]

    def step():
        if args.streams > 1:
            overlapped(parts, sides)
        else:
            step_one_stream()

    sps = timed_steps(step, args.warmup, args.steps, list(ctxs.values()), bsi, stage_timing=False)
    pct = dict(STEP_PERCENTILES)
    sps_one = sps if args.streams == 1 else timed_steps(step_one_stream, 1, args.steps, list(ctxs.values()),
                                                         bsi, stage_timing=False)
    # the same steps again on one stream with the library's stage events, so
    # that every kernel is timed alone
    sps_inst = timed_steps(step_one_stream, 1, args.steps, list(ctxs.values()), bsi)
    STEP_PERCENTILES.clear()
    STEP_PERCENTILES.update(pct)
    stages = {}
    for o in ORDERS:
        stages.update(read_stages(bsi, ctxs[o], f"N{o}"))
        bsi._bsi.bsi_ctx_set_timing(ctxs[o].handle, False)
    eprint(f"{sps * 1e3:.3f} ms/step on {args.streams} stream(s), {sps_one * 1e3:.3f} on one stream, "
           f"{sps_inst * 1e3:.3f} on one stream with stage events")
    print_stages(stages, sps_inst, args.steps)

    # cold last-level cache: the 201 MB grid fits the 256 MB Infinity Cache,
    # so the gather is also timed with a 512 MB buffer written before each call
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    cold = {}
    for o in ORDERS:
        bsi._bsi.bsi_ctx_reset_timing(ctxs[o].handle)
        bsi._bsi.bsi_ctx_set_timing(ctxs[o].handle, True)
        for r in range(10):
            flush.fill_(r + 1)
            fields[o].eval(pos, cfg=cfg, out=outs[o])
        torch.cuda.synchronize()
        cold.update(read_stages(bsi, ctxs[o], f"N{o}", names=("gather",)))
        bsi._bsi.bsi_ctx_set_timing(ctxs[o].handle, False)
    del flush
    copy_gbs = copy_bandwidth()

    U = {o: distinct_stencil_points(pos, N_GRID, o) for o in ORDERS}
    alg = {}
    for k in stages:
        st, o = k.split("@N")
        o = int(o)
        alg[k] = gather_bytes(P, NCOMP, U[o], 4) if st == "gather" else fft_bytes(st, N_GRID, NCOMP, o)
    # dominant kernel: largest share of the step among those with a byte count
    dom = max((k for k in stages if alg[k] is not None), key=lambda k: stages[k]["total_ms"])
    roofline = roofline_entry(dom, alg[dom], stages[dom]["avg_us"], measured_traffic(dom))
    gather_rl = {}
    for o in ORDERS:
        k = f"gather@N{o}"
        if k in stages:
            e = roofline_entry(k, alg[k], stages[k]["avg_us"])
            gather_rl[k] = {"achieved_GBs": e["achieved"], "frac": e["frac"],
                            "frac_of_copy": round(e["achieved"] / copy_gbs, 4),
                            "algorithmic_bytes": alg[k], "distinct_points": U[o], "avg_us": e["avg_us"],
                            "points_per_s": round(P / (stages[k]["avg_us"] * 1e-6), 1)}
            fma_s = P * gather_fma(o, NCOMP) / (stages[k]["avg_us"] * 1e-6)
            gather_rl[k]["alu"] = {"fma_per_particle": gather_fma(o, NCOMP), "achieved_TFMA_s": round(fma_s / 1e12, 3),
                                   "peak_TFMA_s": round(FMA_PEAK_PER_S / 1e12, 3),
                                   "frac": round(fma_s / FMA_PEAK_PER_S, 4)}
            if k in cold:
                c = roofline_entry(k, alg[k], cold[k]["avg_us"])
                gather_rl[k]["cold"] = {"avg_us": c["avg_us"], "achieved_GBs": c["achieved"], "frac": c["frac"],
                                        "frac_of_copy": round(c["achieved"] / copy_gbs, 4)}
    fft_rl = {}
    for k in stages:
        if k.startswith("fft") and alg.get(k):
            e = roofline_entry(k, alg[k], stages[k]["avg_us"], measured_traffic(k))
            fft_rl[k] = {"achieved_GBs": e["achieved"], "frac": e["frac"],
                         "frac_of_copy": round(e["achieved"] / copy_gbs, 4), "algorithmic_bytes": alg[k],
                         "traffic": e["traffic"], "avg_us": e["avg_us"]}
    cpu = None
    if not args.no_cpu_baseline:
        eprint("timing the CPU oracle on a sample ...")
        cpu = cpu_baseline_plain(uhat_np, pos_np, args.cpu_sample)
    for o in ORDERS:
        fields[o].close()
        ctxs[o].close()
    config = {"workload": "256^3 x3 divergence-free Kolmogorov field, FP32 grid, orders 4 and 6, "
                          "1e6 uniform particles; step = prefilter + eval per order",
              "n": N_GRID, "ncomp": NCOMP, "orders": list(ORDERS), "particles": P,
              "grid_dtype": "f32", "spectrum_dtype": "c128", "parallelism": "single GPU"}
    # the prefilter is paid once per snapshot; per order, also the evaluation
    # alone (binning + gather, stage times) and the prefilter alone
    per_order = {}
    for o in ORDERS:
        ev = sum(stages[f"{st}@N{o}"]["avg_us"] for st in EVAL_STAGES if f"{st}@N{o}" in stages)
        pf = sum(stages[f"{st}@N{o}"]["avg_us"] for st in ("fft_axis0", "fft_axis1", "fft_c2r")
                 if f"{st}@N{o}" in stages)
        per_order[f"N{o}"] = {"eval_us": round(ev, 1), "eval_points_per_s": round(P / (ev * 1e-6), 1),
                              "prefilter_us": round(pf, 1)}
    return base_line(args, len(ORDERS) * P / sps, "points/s", sps, "f32", config, roofline, cpu,
                     streams=args.streams, ms_per_step_one_stream=round(sps_one * 1e3, 4),
                     gather_roofline=gather_rl, fft_roofline=fft_rl, per_order=per_order,
                     copy_GBs=round(copy_gbs, 1),
                     stages_us={k: round(v["avg_us"], 2) for k, v in stages.items()})


# ---------------------------------------------------------- hessian form ---

def form_hessian(args):
    """The plain workload with second derivatives: 256^3 x3 FP32 grid, orders 4
    and 6, 10^6 uniform particles; step = prefilter + u, grad u and the six
    second derivatives per component, per order (the orders on two streams)."""
    import torch
    from threadpoolctl import threadpool_limits
    import synth
    import paper_1201_4060_amd as bsi
    dev = torch.device("cuda:0")
    eprint("generating inputs ...")
    uhat_np = synth.kolmogorov_spectrum(N_GRID, NCOMP, seed=FIELD_SEED)
    pos_np = synth.uniform_positions(P, seed=POS_SEED)
    uhat = torch.from_numpy(uhat_np).to(dev)
    pos = torch.from_numpy(pos_np).to(dev)
    ctxs = {o: bsi.Context(0) for o in ORDERS}
    fields = {o: bsi.Field(ctxs[o], N_GRID, NCOMP, o, bsi.BSI_F32) for o in ORDERS}
    outs = {o: (torch.empty((P, NCOMP), dtype=torch.float32, device=dev),
                torch.empty((P, NCOMP, 3), dtype=torch.float32, device=dev),
                torch.empty((P, NCOMP, 6), dtype=torch.float32, device=dev)) for o in ORDERS}

    def order_part(o):
        def run():
            fields[o].set_spectrum(uhat)
            fields[o].eval_hessian(pos, out=outs[o])
        return run

    def step_one_stream():
        for o in ORDERS:
            order_part(o)()

    sides = [torch.cuda.Stream() for _ in ORDERS[1:]]
    parts = [order_part(o) for o in ORDERS]

    def step():
        if args.streams > 1:
            overlapped(parts, sides)
        else:
            step_one_stream()

    sps = timed_steps(step, args.warmup, args.steps, list(ctxs.values()), bsi, stage_timing=False)
    pct = dict(STEP_PERCENTILES)
    sps_inst = timed_steps(step_one_stream, 1, args.steps, list(ctxs.values()), bsi)
    STEP_PERCENTILES.clear()
    STEP_PERCENTILES.update(pct)
    stages = {}
    for o in ORDERS:
        stages.update(read_stages(bsi, ctxs[o], f"N{o}", names=STAGES + ("hess_items", "gather_hess")))
        bsi._bsi.bsi_ctx_set_timing(ctxs[o].handle, False)
    eprint(f"{sps * 1e3:.3f} ms/step on {args.streams} stream(s), {sps_inst * 1e3:.3f} on one stream "
           f"with stage events")
    print_stages(stages, sps_inst, args.steps)
    U = {o: distinct_stencil_points(pos, N_GRID, o) for o in ORDERS}
    alg = {}
    for k in stages:
        st, o = k.split("@N")
        o = int(o)
        if st == "gather_hess":
            # positions in; u, grad u and six second derivatives out (10 C values)
            alg[k] = P * (24 + 10 * NCOMP * 4) + U[o] * NCOMP * 4
        else:
            alg[k] = fft_bytes(st, N_GRID, NCOMP, o)
    dom = max((k for k in stages if alg[k] is not None), key=lambda k: stages[k]["total_ms"])
    roofline = roofline_entry(dom, alg[dom], stages[dom]["avg_us"])
    hess_rl = {}
    for o in ORDERS:
        k = f"gather_hess@N{o}"
        e = roofline_entry(k, alg[k], stages[k]["avg_us"])
        fma_s = P * hessian_fma(o, NCOMP) / (stages[k]["avg_us"] * 1e-6)
        hess_rl[k] = {"achieved_GBs": e["achieved"], "frac": e["frac"], "avg_us": e["avg_us"],
                      "algorithmic_bytes": alg[k], "fma_per_particle": hessian_fma(o, NCOMP),
                      "alu_frac": round(fma_s / FMA_PEAK_PER_S, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sample = 20000
        idx = np.random.default_rng(0).choice(P, sample, replace=False)
        total = 0.0
        with threadpool_limits(limits=1):
            for o in ORDERS:
                t0 = time.perf_counter()
                grid = oracle.prefilter(uhat_np, o)
                t1 = time.perf_counter()
                oracle.evaluate_hessian(grid, pos_np[idx], o)
                t2 = time.perf_counter()
                del grid
                total += (t1 - t0) + (t2 - t1) * (P / sample)
                eprint(f"cpu oracle order {o}: prefilter {t1 - t0:.2f} s, hessian of {sample} particles "
                       f"{t2 - t1:.2f} s")
        cpu = {"value": len(ORDERS) * P / total, "unit": "points/s", "cores": 1, "kind": "oracle",
               "sample": (f"full FP64 prefilter of the 256^3x3 field per order + u, grad u and second "
                          f"derivatives of {sample} of the 1e6 particles per order, scaled to 1e6; numpy, "
                          f"one thread")}
    for o in ORDERS:
        fields[o].close()
        ctxs[o].close()
    config = {"workload": "256^3 x3 divergence-free Kolmogorov field, FP32 grid, orders 4 and 6, 1e6 uniform "
                          "particles; step = prefilter + u, grad u and second derivatives per order",
              "n": N_GRID, "ncomp": NCOMP, "orders": list(ORDERS), "particles": P, "grid_dtype": "f32",
              "outputs": "u, grad u, hessian (6 per component)", "parallelism": "single GPU"}
    return base_line(args, len(ORDERS) * P / sps, "points/s", sps, "f32", config, roofline, cpu,
                     streams=args.streams, hessian_roofline=hess_rl,
                     stages_us={k: round(v["avg_us"], 2) for k, v in stages.items()})


# -------------------------------------------------------- precision form ---

PREC_N, PREC_C, PREC_ORDER, PREC_P = 512, 3, 6, 10_000_000
PREC_FIELD_SEED, PREC_POS_SEED = 2, 102
PREC_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_512cube_x3_order6_1e7_clustered.md")


def _oracle_component_prefilter(args):
    # one component of the FP64 prefilter, written into shared memory
    from multiprocessing import shared_memory
    import oracle
    shm_name, c, N, shape = args
    uhat = _CPU_SHARED["uhat"]
    t0 = time.perf_counter()
    g = oracle.prefilter(uhat[c:c + 1], N)[0]
    t1 = time.perf_counter()
    shm = shared_memory.SharedMemory(name=shm_name)
    out = np.ndarray(shape, dtype=np.float64, buffer=shm.buf)
    out[c] = g
    del out
    shm.close()
    return t1 - t0


def _oracle_eval_chunk(args):
    import oracle
    lo, hi, N = args
    t0 = time.perf_counter()
    oracle.evaluate(_CPU_SHARED["grid"], _CPU_SHARED["pos"][lo:hi], N)
    return time.perf_counter() - t0


_CPU_SHARED = {}


def cpu_baseline_all_cores(uhat, pos, N, P_total, per_worker, workers, label):
    """The FP64 oracle as it stands, timed on the host's cores: its prefilter
    with one process per field component, then its evaluation of a bounded
    particle sample split over `workers` processes (fork; each numpy call
    single-threaded); the sample's rate is scaled to the whole particle set.
    Also reports the same work on one thread (component prefilter times summed,
    a smaller sample evaluated alone)."""
    import multiprocessing as mp
    from multiprocessing import shared_memory
    from threadpoolctl import threadpool_limits
    import oracle
    C = uhat.shape[0]
    n = uhat.shape[1]
    shape = (C, n, n, n)
    shm = shared_memory.SharedMemory(create=True, size=int(np.prod(shape)) * 8)
    try:
        _CPU_SHARED["uhat"] = uhat
        ctx = mp.get_context("fork")
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            with ctx.Pool(C) as pool:
                comp_times = pool.map(_oracle_component_prefilter, [(shm.name, c, N, shape) for c in range(C)])
            t_pf = time.perf_counter() - t0
            grid = np.ndarray(shape, dtype=np.float64, buffer=shm.buf)
            rng = np.random.default_rng(0)
            sample = np.sort(rng.choice(pos.shape[0], per_worker * workers, replace=False))
            _CPU_SHARED["grid"] = grid
            _CPU_SHARED["pos"] = np.ascontiguousarray(pos[sample])
            chunks = [(w * per_worker, (w + 1) * per_worker, N) for w in range(workers)]
            t1 = time.perf_counter()
            with ctx.Pool(workers) as pool:
                pool.map(_oracle_eval_chunk, chunks)
            t_ev = time.perf_counter() - t1
            # one thread: a smaller sample evaluated in this process
            one = min(per_worker, 20000)
            t2 = time.perf_counter()
            oracle.evaluate(grid, _CPU_SHARED["pos"][:one], N)
            t_one = time.perf_counter() - t2
            del grid
    finally:
        _CPU_SHARED.clear()
        shm.close()
        shm.unlink()
    S = per_worker * workers
    total = t_pf + t_ev * P_total / S
    total_one = sum(comp_times) + t_one * P_total / one
    try:
        model = next(ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name"))
    except (OSError, StopIteration):
        model = "unknown"
    eprint(f"cpu oracle: prefilter {t_pf:.2f} s on {C} processes (components {comp_times}), "
           f"eval of {S} particles {t_ev:.2f} s on {workers} processes; one thread: eval {one} in {t_one:.2f} s")
    return {"value": P_total / total, "unit": "points/s", "cores": max(workers, C), "kind": "oracle",
            "sample": (f"FP64 oracle prefilter of the {label} field (one process per component, "
                       f"{t_pf:.1f} s) + evaluation of {S} of the {P_total} particles on {workers} processes "
                       f"({t_ev:.1f} s), scaled to all particles; numpy, one thread per process"),
            "host": {"nproc": os.cpu_count(), "model": model},
            "one_thread": {"value": P_total / total_one, "unit": "points/s",
                           "sample": f"component prefilters summed ({sum(comp_times):.1f} s) + {one} particles "
                                     f"evaluated on one thread ({t_one:.2f} s), scaled"}}


def form_precision(args):
    """512^3 x3 divergence-free field, order 6, 10^7 clustered particles (5e6
    uniform + 100 Gaussian blobs of 5e4, sigma 0.1).  The headline step is the
    FP32-grid path (prefilter + binning + gather); the BF16-grid path and the
    plain FP64-grid path run the same step on the same inputs, timed apart;
    every path's error against the FP64 oracle is reported on a sample."""
    import torch
    import synth
    import oracle
    import paper_1201_4060_amd as bsi
    n, C, N, Pp = PREC_N, PREC_C, PREC_ORDER, PREC_P
    eprint("generating the 512^3 spectrum and 1e7 clustered particles ...")
    uhat_np = synth.kolmogorov_spectrum(n, C, seed=PREC_FIELD_SEED)
    pos_np = synth.clustered_positions(5_000_000, 100, 50_000, 0.1, seed=PREC_POS_SEED)
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is touched: the oracle's worker processes are forked
        eprint("timing the CPU oracle on the host's cores ...")
        workers = max(1, min(args.cpu_workers, os.cpu_count() or 1))
        cpu = cpu_baseline_all_cores(uhat_np, pos_np, N, Pp, args.cpu_per_worker, workers, "512^3x3")
    dev = torch.device("cuda:0")
    kinds = (("f32", bsi.BSI_F32, 4), ("bf16", bsi.BSI_BF16, 2), ("f64", bsi.BSI_F64, 8))
    ctxs = {k: bsi.Context(0) for k, _, _ in kinds}
    uhat = torch.from_numpy(uhat_np).to(dev)
    pos = torch.from_numpy(pos_np).to(dev)
    fields = {k: bsi.Field(ctxs[k], n, C, N, dt) for k, dt, _ in kinds}
    outs = {k: (torch.empty((Pp, C), dtype=fields[k].out_dtype, device=dev),
                torch.empty((Pp, C, 3), dtype=fields[k].out_dtype, device=dev)) for k, _, _ in kinds}

    def part(k):
        def run():
            fields[k].set_spectrum(uhat)
            fields[k].eval(pos, out=outs[k])
        return run

    sps, pct, stages = {}, {}, {}
    for k, _, _ in kinds:
        steps = args.steps if k != "f64" else max(2, args.steps // 2)
        sps[k] = timed_steps(part(k), args.warmup, steps, [ctxs[k]], bsi, stage_timing=False)
        pct[k] = dict(STEP_PERCENTILES)
        timed_steps(part(k), 1, steps, [ctxs[k]], bsi)   # the same steps with the library's stage events
        stages.update(read_stages(bsi, ctxs[k], k))
        bsi._bsi.bsi_ctx_set_timing(ctxs[k].handle, False)
        eprint(f"{k}: {sps[k] * 1e3:.3f} ms/step")
    STEP_PERCENTILES.clear()
    STEP_PERCENTILES.update(pct["f32"])
    print_stages({s: v for s, v in stages.items() if s.endswith("@f32")}, sps["f32"], args.steps)
    copy_gbs = copy_bandwidth()
    U = distinct_stencil_points(pos, n, N)
    cbytes = {k: cb for k, _, cb in kinds}
    obytes = {"f32": 4, "bf16": 4, "f64": 8}
    alg = {}
    for key in stages:
        st, k = key.split("@")
        if st == "gather":
            alg[key] = gather_bytes(Pp, C, U, cbytes[k], obytes[k])
        else:
            alg[key] = fft_bytes(st, n, C, N, grid_bytes=cbytes[k], work_bytes=16 if k == "f64" else 8)
    # FP64 vector FMA runs at the unpacked FP32 rate on this chip (78.6 TFLOP/s)
    fma_peak = {"f32": FMA_PEAK_PER_S, "bf16": FMA_PEAK_PER_S, "f64": FMA_PEAK_PER_S}

    def gather_entry(k):
        key = f"gather@{k}"
        e = roofline_entry(key, alg[key], stages[key]["avg_us"], measured_traffic(key, PREC_TRAFFIC_FILE))
        fma_s = Pp * gather_fma(N, C) / (stages[key]["avg_us"] * 1e-6)
        e["frac_of_copy"] = round(e["achieved"] / copy_gbs, 4)
        e["alu"] = {"fma_per_particle": gather_fma(N, C), "achieved_TFMA_s": round(fma_s / 1e12, 3),
                    "peak_TFMA_s": round(fma_peak[k] / 1e12, 3), "frac": round(fma_s / fma_peak[k], 4)}
        e["points_per_s"] = round(Pp / (stages[key]["avg_us"] * 1e-6), 1)
        return e

    roofline = gather_entry("f32")
    legs = {}
    for k, _, _ in kinds:
        ev = sum(stages[f"{st}@{k}"]["avg_us"] for st in EVAL_STAGES if f"{st}@{k}" in stages)
        pf = sum(stages[f"{st}@{k}"]["avg_us"] for st in ("fft_axis0", "fft_axis1", "fft_c2r"))
        legs[k] = {"points_per_s": round(Pp / sps[k], 1), "ms_per_step": round(sps[k] * 1e3, 4),
                   "ms_per_step_percentiles": pct[k], "prefilter_us": round(pf, 1), "eval_us": round(ev, 1),
                   "eval_points_per_s": round(Pp / (ev * 1e-6), 1), "grid_bytes": fields[k].nbytes(),
                   "gather": gather_entry(k) if k != "f32" else "see roofline",
                   "stages_us": {s.split("@")[0]: round(v["avg_us"], 2) for s, v in stages.items()
                                 if s.endswith("@" + k)}}
    # errors of every path against the FP64 oracle on a particle sample
    # (outside the timed region); the oracle's grid comes from its own prefilter
    eprint("FP64 oracle on a sample ...")
    sample = np.sort(np.random.default_rng(1).choice(Pp, args.cpu_sample_precision, replace=False))
    grid = oracle.prefilter(uhat_np, N)
    want_u, want_g = oracle.evaluate(grid, pos_np[sample], N)
    umax = float(np.abs(grid).max())
    del grid
    S6 = 115.0 / 96.0  # max_t sum_j |w'_j(t)| of the order-6 derivative weights
    idx = torch.from_numpy(sample).to(dev)
    for k, _, _ in kinds:
        u = outs[k][0][idx].double().cpu().numpy()
        g = outs[k][1][idx].double().cpu().numpy()
        errs = {}
        for name, got, want in (("u", u, want_u), ("grad", g, want_g)):
            got = got.reshape(got.shape[0], -1)
            want = want.reshape(want.shape[0], -1)
            scale = np.abs(want).max(axis=0)
            d = np.abs(got - want)
            pointwise = d / np.maximum(np.abs(want), 1e-3 * scale)
            errs[name] = {"max_rel": float((d.max(axis=0) / scale).max()),
                          "rms_rel": float((np.sqrt((d ** 2).mean(axis=0)) /
                                            np.sqrt((want ** 2).mean(axis=0))).max()),
                          "p99_pointwise_rel": float(np.percentile(pointwise, 99))}
        if k == "bf16":
            errs["bound_u_abs"] = 2.0 ** -8 * umax
            errs["bound_grad_abs"] = 2.0 ** -8 * umax * S6 * n / (2 * np.pi)
            errs["max_abs_u"] = float(np.abs(u - want_u).max())
            errs["max_abs_grad"] = float(np.abs(g - want_g).max())
        legs[k]["error_vs_fp64_oracle"] = errs
        eprint(f"  {k}: {json.dumps(errs)}")
    for k, _, _ in kinds:
        fields[k].close()
        ctxs[k].close()
    del outs
    methods = None
    if args.methods_in_default:
        methods = methods_legs(bsi, uhat, pos, n, C, args)
    del uhat, pos, uhat_np
    torch.cuda.empty_cache()
    config = {"workload": "512^3 x3 divergence-free Kolmogorov field, order 6, 1e7 clustered particles "
                          "(5e6 uniform + 100 Gaussian blobs of 5e4, sigma 0.1); step = prefilter (FP64 symbol "
                          "multiply + inverse 3D real FFT) + binning + gather of u and grad u; headline: FP32 "
                          "coefficient grid; the BF16-grid and FP64-grid paths timed on the same inputs",
              "n": n, "ncomp": C, "order": N, "particles": Pp, "grid_dtype": "f32", "spectrum_dtype": "c128",
              "parallelism": "single GPU"}
    extra = {"legs": legs, "copy_GBs": round(copy_gbs, 1)}
    if methods is not None:
        extra["methods"] = methods
    if args.serve_in_default:
        extra["serving"] = serve_summary(args)
    return base_line(args, Pp / sps["f32"], "points/s", sps["f32"], "f32", config, roofline, cpu, **extra)


# ---------------------------------------------------------- methods leg ---

# (name, basis, order, prefilter) of the four methods of Table 2 (and the
# order-6 B-spline of the headline), all on FP32 grids
METHODS = (("bspline4", "BSPLINE", 4, "L2OPT"), ("bspline6", "BSPLINE", 6, "L2OPT"),
           ("lagrange4", "LAGRANGE", 4, "NONE"), ("lagrange6", "LAGRANGE", 6, "NONE"),
           ("linear", "LAGRANGE", 2, "NONE"), ("hermite", "HERMITE", 4, "NONE"))


def methods_legs(bsi, uhat, pos, n, C, args):
    """The methods Table 2 compares, on the same spectrum and particles, FP32
    grids: per method the prefilter (B-spline: one inverse FFT per component;
    Lagrange and linear: one FFT with c = 1; Hermite: eight, one per
    derivative field) and the evaluation (binning + gather), timed by the
    library's stage events over `steps` steps of set_spectrum + eval."""
    import torch
    P_ = pos.shape[0]
    ctx = bsi.Context(0)
    out = {}
    steps = max(3, args.steps // 2)
    for name, basis, N, pf in METHODS:
        f = bsi.Field(ctx, n, C, N, bsi.BSI_F32, prefilter=getattr(bsi, "BSI_PREFILTER_" + pf),
                      basis=getattr(bsi, "BSI_BASIS_" + basis))
        u = torch.empty((P_, C), dtype=torch.float32, device=pos.device)
        g = torch.empty((P_, C, 3), dtype=torch.float32, device=pos.device)

        def step():
            f.set_spectrum(uhat)
            f.eval(pos, out=(u, g))

        sec = timed_steps(step, 1, steps, [ctx], bsi)
        st = read_stages(bsi, ctx, name)
        bsi._bsi.bsi_ctx_set_timing(ctx.handle, False)
        per = {k.split("@")[0]: v["total_ms"] * 1e3 / steps for k, v in st.items()}
        pf_us = sum(per.get(s, 0.0) for s in ("fft_axis0", "fft_axis1", "fft_c2r"))
        ev_us = sum(per.get(s, 0.0) for s in EVAL_STAGES)
        launches = {k.split("@")[0]: st[k]["launches"] // steps for k in st
                    if k.split("@")[0] in ("fft_axis0", "fft_axis1", "fft_c2r")}
        fields = 8 if basis == "HERMITE" else 1
        out[name] = {"basis": basis.lower(), "order": N, "prefilter": pf.lower(),
                     "inverse_ffts_per_component": fields, "pass_launches_per_step": launches,
                     "grid_bytes": f.nbytes(),
                     "prefilter_us": round(pf_us, 1), "eval_us": round(ev_us, 1),
                     "gather_us": round(per.get("gather", 0.0), 1),
                     "eval_points_per_s": round(P_ / (ev_us * 1e-6), 1),
                     "ms_per_step": round(sec * 1e3, 4), "points_per_s": round(P_ / sec, 1)}
        eprint(f"{name}: prefilter {pf_us:.1f} us ({fields} inverse FFTs, passes {launches}), "
               f"eval {ev_us:.1f} us, {sec * 1e3:.3f} ms/step")
        f.close()
        del u, g
    ctx.close()
    torch.cuda.empty_cache()
    out["hermite_vs_bspline4_prefilter"] = round(out["hermite"]["prefilter_us"] / out["bspline4"]["prefilter_us"], 2)
    out["note"] = ("FP32 grids, same spectrum and particles as the headline; inverse FFTs per component are "
                   "the method's count (Table 2); one launch of each pass transforms all components, and the "
                   "Hermite fields of axis-2 orders 0 and 1 share their axis-0/1 passes and one axis-2 pass; "
                   "stage times are per step")
    return out


def form_methods(args):
    """The methods leg alone on the 512^3 x3 workload (see methods_legs)."""
    import torch
    import synth
    import paper_1201_4060_amd as bsi
    n, C = PREC_N, PREC_C
    uhat = torch.from_numpy(synth.kolmogorov_spectrum(n, C, seed=PREC_FIELD_SEED)).to("cuda:0")
    pos = torch.from_numpy(synth.clustered_positions(5_000_000, 100, 50_000, 0.1, seed=PREC_POS_SEED)).to("cuda:0")
    m = methods_legs(bsi, uhat, pos, n, C, args)
    b = m["bspline4"]
    config = {"workload": "512^3 x3 divergence-free Kolmogorov field, 1e7 clustered particles; the methods of "
                          "Table 2 on FP32 grids; value: the order-4 B-spline step",
              "n": n, "ncomp": C, "particles": pos.shape[0], "parallelism": "single GPU"}
    return base_line(args, b["points_per_s"], "points/s", b["ms_per_step"] * 1e-3, "f32", config, None, None,
                     methods=m)


# ------------------------------------------------------------ batch form ---

def batch_specs(count=64):
    """Field f: n uniform over {64,128,192,256}, order uniform over {4,6},
    P = round(10^U(3,6)); draws from stream 13 of seed 300+f."""
    from synth.rng import keyed_uniform
    specs = []
    for f in range(count):
        u = keyed_uniform(300 + f, 13, np.arange(3))
        n = (64, 128, 192, 256)[min(int(u[0] * 4), 3)]
        N = (4, 6)[min(int(u[1] * 2), 1)]
        Pf = int(round(10 ** (3 + 3 * u[2])))
        specs.append((n, N, Pf))
    return specs


def form_batch(args):
    import torch
    from threadpoolctl import threadpool_limits
    import synth
    import oracle
    import paper_1201_4060_amd as bsi
    dev = torch.device("cuda:0")
    specs = batch_specs()
    ctx = bsi.Context(0)
    fields, items = [], []
    eprint("building 64 fields ...")
    spec_buf = {}
    for f, (n, N, Pf) in enumerate(specs):
        if n not in spec_buf:
            spec_buf[n] = torch.empty((3, n, n, n // 2 + 1), dtype=torch.complex128, device=dev)
        bsi._bsi.bsi_synth_kolmogorov(ctx.handle, n, 3, 300 + f, spec_buf[n])
        fld = bsi.Field(ctx, n, 3, N, bsi.BSI_F32)
        fld.set_spectrum(spec_buf[n])
        pos = torch.from_numpy(synth.uniform_positions(Pf, seed=400 + f)).to(dev)
        u = torch.empty((Pf, 3), dtype=torch.float32, device=dev)
        g = torch.empty((Pf, 3, 3), dtype=torch.float32, device=dev)
        fields.append(fld)
        items.append((fld, pos, u, g))
    del spec_buf
    torch.cuda.synchronize()
    Ptot = sum(s[2] for s in specs)
    eprint(f"{Ptot} particles in total; autotuning ...")
    tuned = set()
    t0 = time.perf_counter()
    for (n, N, Pf), fld in zip(specs, fields):
        key = (N, round(np.log2(Pf / n ** 3)))
        if key not in tuned:
            tuned.add(key)
            bsi._bsi.bsi_tune(fld.handle, Pf, seed=len(tuned))
    eprint(f"  {len(tuned)} tuning runs in {time.perf_counter() - t0:.1f} s")
    batch = bsi.Batch(ctx, items)
    modes = [batch.item_config(i) for i in range(len(items))]
    n_tiled = sum(1 for c in modes if c.variant == 0)

    # the figure of the line: graph replays without the library's stage events
    sps = timed_steps(lambda: batch.run(use_graph=True), args.warmup, args.steps, [ctx], bsi,
                      stage_timing=False)
    graph_pct = dict(STEP_PERCENTILES)
    timed_steps(lambda: batch.run(use_graph=True), 1, args.steps, [ctx], bsi)
    graph = read_stages(bsi, ctx, "graph", ("batch_graph",))
    # the same batch enqueued directly, for the per-kernel times
    sps_eager = timed_steps(lambda: batch.run(use_graph=False), 1, args.steps, [ctx], bsi)
    st_eager = read_stages(bsi, ctx, "batch", ("batch_bin", "batch_gather"))
    # one launch sequence per field with the same configurations, for comparison
    cfgs = [bsi._bsi.bsi_ctx_lookup_config(ctx.handle, fl.handle, it[1].shape[0])
            for fl, it in zip(fields, items)]

    def singles():
        for (fl, pos, u, g), c in zip(items, cfgs):
            fl.eval(pos, cfg=c, out=(u, g))

    sps_single = timed_steps(singles, 1, args.steps, [ctx], bsi, stage_timing=False)
    timed_steps(singles, 1, args.steps, [ctx], bsi)
    st_single = read_stages(bsi, ctx, "single", ("gather",))
    bsi._bsi.bsi_ctx_set_timing(ctx.handle, False)
    stages = {**graph, **st_eager, **st_single}
    print_stages(stages, sps, args.steps)
    eprint(f"graph {sps * 1e3:.3f} ms/step, direct {sps_eager * 1e3:.3f}, per-field launches "
           f"{sps_single * 1e3:.3f}")
    mark = torch.zeros(256 ** 3, dtype=torch.bool, device=dev)
    alg = 0
    for (n, N, Pf), (fl, pos, u, g) in zip(specs, items):
        alg += gather_bytes(Pf, 3, distinct_stencil_points(pos, n, N, mark[: n ** 3]), 4)
    del mark
    roofline = roofline_entry("batch_gather", alg, stages["batch_gather@batch"]["avg_us"])
    # CPU baseline: the oracle evaluating a sample of three fields (n = 64, 128, 192)
    cpu = None
    if not args.no_cpu_baseline:
        eprint("timing the CPU oracle on a sample ...")
        done, t_eval, pts = set(), 0.0, 0
        with threadpool_limits(limits=1):
            for f, (n, N, Pf) in enumerate(specs):
                if n in done or n > 192:
                    continue
                done.add(n)
                grid = oracle.prefilter(synth.kolmogorov_spectrum(n, 3, seed=300 + f), N)
                m = min(Pf, 20000)
                p = synth.uniform_positions(Pf, seed=400 + f)[:m]
                t0 = time.perf_counter()
                oracle.evaluate(grid, p, N)
                t_eval += time.perf_counter() - t0
                pts += m
        cpu = {"value": pts / t_eval, "unit": "points/s", "cores": 1, "kind": "oracle",
               "sample": (f"oracle evaluation of {pts} particles of the first fields with n = 64, 128, "
                          f"192 (grids from the oracle's prefilter, not timed); numpy, one thread")}
    batch.close()
    for fl in fields:
        fl.close()
    ctx.close()
    config = {"workload": "64 divergence-free Kolmogorov fields, n uniform over {64,128,192,256}, order "
                          "uniform over {4,6}, FP32 grids, 10^U(3,6) uniform particles each; step = one "
                          "replay of the captured graph (binning, then per (order, components) class a persistent tile "
                          "gather and a direct gather launch)",
              "fields": len(specs), "particles": Ptot, "tiled_items": n_tiled,
              "direct_items": len(specs) - n_tiled, "tuning_runs": len(tuned), "parallelism": "single GPU"}
    STEP_PERCENTILES.clear()
    STEP_PERCENTILES.update(graph_pct)   # the step the line reports: the graph replay
    return base_line(args, Ptot / sps, "points/s", sps, "f32", config, roofline, cpu,
                     direct_enqueue_points_per_s=round(Ptot / sps_eager, 1),
                     per_field_launches_points_per_s=round(Ptot / sps_single, 1),
                     stages_us={k: round(v["avg_us"], 2) for k, v in stages.items()})


# ------------------------------------------------------------ serve form ---

def serve_run(args, nreq):
    """Resident snapshots served to Poisson particle-query requests: the saturated
    closed-loop rate R, then open loop at 0.5 R and 0.8 R (nreq requests each)."""
    import torch
    import synth
    import paper_1201_4060_amd as bsi
    from synth.rng import keyed_uniform
    dev = torch.device("cuda:0")
    big_n, n_big, small_n, n_small = (1024, 8, 256, 32) if args.serve_scale == "full" else (512, 2, 128, 8)
    ctx = bsi.Context(0)
    fields = {}
    eprint(f"building {n_big} x {big_n}^3 + {n_small} x {small_n}^3 resident snapshots, orders 4 and 6 ...")
    t0 = time.perf_counter()
    snap = 0
    for n, count, prec in ((big_n, n_big, torch.complex64), (small_n, n_small, torch.complex128)):
        spec = torch.empty((3, n, n, n // 2 + 1), dtype=prec, device=dev)
        for _ in range(count):
            bsi._bsi.bsi_synth_kolmogorov(ctx.handle, n, 3, 500 + snap, spec)
            for N in (4, 6):
                fl = bsi.Field(ctx, n, 3, N, bsi.BSI_F32)
                fl.set_spectrum(spec)
                fields[2 * snap + (N == 6)] = fl
            snap += 1
            eprint(f"  snapshot {snap} ready ({time.perf_counter() - t0:.1f} s)")
        del spec
        torch.cuda.synchronize()
        bsi._bsi.bsi_ctx_trim(ctx.handle)
        torch.cuda.empty_cache()
    resident = sum(f.nbytes() for f in fields.values())
    eprint(f"{len(fields)} resident grids, {resident / 2**30:.1f} GiB")
    # request positions: slices of a uniform and a clustered pool
    pool_n = 2_000_000
    pools = []
    for p in (synth.uniform_positions(pool_n, seed=600),
              synth.clustered_positions(pool_n // 2, 100, pool_n // 200, 0.1, seed=601)):
        t = torch.empty((pool_n, 3), dtype=torch.float64, pin_memory=True)
        t.numpy()[:] = p
        pools.append(t)
    nbuf = 48
    maxp = 1_000_000
    outs = [(torch.empty((maxp, 3), dtype=torch.float32, pin_memory=True),
             torch.empty((maxp, 3, 3), dtype=torch.float32, pin_memory=True)) for _ in range(nbuf)]
    nsnap = n_big + n_small

    def request(i):
        u = keyed_uniform(600, 14, np.arange(5 * i, 5 * i + 5))
        s = min(int(u[0] * nsnap), nsnap - 1)
        N6 = int(u[1] >= 0.5)
        Pr = int(round(10 ** (3 + 3 * u[2])))
        pool = pools[1 if u[3] >= 0.5 else 0]
        off = min(int(u[4] * (pool_n - Pr)), pool_n - Pr)
        return 2 * s + N6, pool[off: off + Pr], Pr

    sv = bsi.Server(ctx, hbm_budget=args.serve_budget << 20, max_slots=args.serve_slots)
    for fid, fl in fields.items():
        sv.add_field(fid, fl)

    def run(nreq, start, rate=None, closed=None):
        """Submit requests start..start+nreq-1: Poisson arrivals at `rate`
        requests/s, or closed loop with `closed` outstanding requests."""
        tickets = []
        collected = set()

        def collect(t):
            # a ticket's results are collected once (a second wait is an error)
            if t not in collected:
                sv.wait(t)
                collected.add(t)

        rng = np.random.default_rng(start)
        t_next = time.perf_counter()
        for i in range(nreq):
            j = len(tickets)
            if j >= nbuf:                      # output buffer reuse
                collect(tickets[j - nbuf])
            if closed is not None and j >= closed:
                collect(tickets[j - closed])
            if rate is not None:
                t_next += rng.exponential(1.0 / rate)
                while time.perf_counter() < t_next:
                    pass
            fid, pos, Pr = request(start + i)
            u, g = outs[j % nbuf]
            tickets.append(sv.submit(fid, pos, u[:Pr], g[:Pr]))
        for t in tickets:
            collect(t)
        return sv.stats()

    eprint("warm-up ...")
    run(64, 0, closed=16)
    sv.reset_stats()
    eprint("closed loop (16 outstanding) ...")
    t0 = time.perf_counter()
    sat = run(nreq, 1000, closed=16)
    wall = time.perf_counter() - t0
    R = sat["completed"] / wall
    results = {"saturated": {"requests_per_s": round(R, 1), "points_per_s": round(sat["points_per_s"], 1),
                             "p50_ms": sat["p50_ns"] / 1e6, "p99_ms": sat["p99_ns"] / 1e6,
                             "max_inflight": sat["max_inflight"]}}
    eprint(f"  {R:.0f} requests/s, {sat['points_per_s']:.3e} points/s")
    for frac in (0.5, 0.8):
        sv.reset_stats()
        eprint(f"open loop at {frac} x saturated rate ...")
        st = run(nreq, 100000 * int(10 * frac), rate=frac * R)
        results[f"rate_{frac}"] = {"rate_req_s": round(frac * R, 1), "points_per_s": round(st["points_per_s"], 1),
                                   "p50_ms": st["p50_ns"] / 1e6, "p99_ms": st["p99_ns"] / 1e6,
                                   "device_p50_ms": st["device_p50_ns"] / 1e6,
                                   "device_p99_ms": st["device_p99_ns"] / 1e6,
                                   "max_inflight": st["max_inflight"],
                                   "peak_arena_MiB": round(st["peak_arena_bytes"] / 2**20, 1)}
        eprint(f"  {json.dumps(results[f'rate_{frac}'])}")
    sv.close()
    for fl in fields.values():
        fl.close()
    ctx.close()
    config = {"workload": f"{n_big} x {big_n}^3 + {n_small} x {small_n}^3 resident divergence-free Kolmogorov "
                          "snapshots, FP32 grids for orders 4 and 6; Poisson requests (snapshot uniform, order "
                          "uniform, 10^U(3,6) particles, half uniform / half clustered positions) from pinned "
                          "host memory; value at 0.8 x the saturated request rate",
              "resident_GiB": round(resident / 2**30, 1), "requests_per_run": nreq,
              "slots": args.serve_slots, "hbm_budget_MiB": args.serve_budget, "parallelism": "single GPU"}
    return results, config


def form_serve(args):
    results, config = serve_run(args, args.serve_requests)
    main_rate = results["rate_0.8"]
    line = base_line(args, main_rate["points_per_s"], "points/s", 0.0, "f32", config, None, None,
                     serving=results, p50_ms=main_rate["p50_ms"], p99_ms=main_rate["p99_ms"])
    line["steps"] = args.serve_requests
    line["ms_per_step"] = round(1e3 / main_rate["rate_req_s"], 4) if main_rate["rate_req_s"] else None
    return line


def serve_summary(args):
    """The serving form attached to the headline line: p50 / p99 latency at
    0.5 and 0.8 of the saturated request rate (fewer requests than --form serve)."""
    import torch
    eprint("serving leg ...")
    results, config = serve_run(args, args.serve_requests_default)
    torch.cuda.empty_cache()
    return {"workload": config["workload"], "resident_GiB": config["resident_GiB"],
            "requests_per_run": config["requests_per_run"], "results": results,
            "p50_ms_at_0.8R": results["rate_0.8"]["p50_ms"], "p99_ms_at_0.8R": results["rate_0.8"]["p99_ms"]}


# ------------------------------------------------------------ copy form ---

def copy_calibration(steps):
    """Plain device copy of a known size: the yardstick for HBM byte counters.

    Copies a 1 GiB FP32 buffer `steps` times; each launch reads and writes
    exactly 2^30 bytes, so FETCH_SIZE / WRITE_SIZE of this kernel give the
    factor that turns those counters into bytes for the library's kernels.
    """
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"form": "copy", "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes,
            "launches": steps, "GBs_read_plus_write": round(2 * nbytes / dt / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--form", choices=("plain", "precision", "batch", "serve", "hessian", "methods", "copy"),
                    default="precision")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=100000)
    ap.add_argument("--cpu-sample-precision", type=int, default=100000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sort-tile", type=int, default=None)
    ap.add_argument("--streams", type=int, choices=(1, 2), default=2,
                    help="plain and precision forms: run the two independent halves of a step on 1 or 2 streams")
    ap.add_argument("--serve-scale", choices=("full", "small"), default="full")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget", type=int, default=8192, help="server arena in MiB")
    ap.add_argument("--serve-requests-default", type=int, default=1000,
                    help="requests per rate point of the serving leg attached to the precision form")
    ap.add_argument("--no-serve", dest="serve_in_default", action="store_false",
                    help="precision form: skip the attached serving leg")
    ap.add_argument("--no-methods", dest="methods_in_default", action="store_false",
                    help="precision form: skip the attached methods leg (Table 2's methods timed)")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="host processes of the CPU oracle baseline (capped at the CPU count)")
    ap.add_argument("--cpu-per-worker", type=int, default=25000,
                    help="particles each oracle process evaluates in the CPU baseline")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        eprint("bench.py measures one GPU only: the interpolation of one field runs on a single "
               "MI355X here; multi-GPU sharding (slabs + all-to-all transposes) is not built. "
               "Run with --gpus 1.")
        sys.exit(2)
    if args.form == "copy":
        print(json.dumps(copy_calibration(max(args.steps, 1))), flush=True)
        return
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    form = {"plain": form_plain, "precision": form_precision, "batch": form_batch, "serve": form_serve,
            "hessian": form_hessian, "methods": form_methods}
    print(json.dumps(form[args.form](args)), flush=True)


if __name__ == "__main__":
    main()
