#!/usr/bin/env python3
"""Throughput benchmark of the B-spline interpolation hot path on one MI355X.

Workload: a 256^3 three-component divergence-free Kolmogorov field (spectrum
|uhat|^2 ~ k^-11/3, cut-off |k| <= n/3, complex128 input), FP32 coefficient
grid, spline orders 4 and 6, 10^6 uniform particles.  One step runs the whole
path for each order: prefilter (FP64 symbol multiply + inverse 3D real FFT)
then evaluation (cell/Morton binning + gather) of u and grad u at every
particle.  value = interpolated points (particles x orders) per second of
whole step, inputs resident in HBM.

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
STAGES = ("fft_axis0", "fft_axis1", "fft_c2r", "bin_count", "bin_scan", "bin_scatter", "gather")


def eprint(*a):
    print(*a, file=sys.stderr, flush=True)


def distinct_stencil_points(pos, n, order):
    """Number of distinct grid points in the union of all particles' stencils."""
    h = 2.0 * np.pi / n
    cell = np.mod(np.floor(pos * (n / (2.0 * np.pi))).astype(np.int64), n)
    mark = np.zeros(n * n * n, dtype=bool)
    offs = np.arange(order) - order // 2 + 1
    for a in offs:
        i0 = np.mod(cell[:, 0] + a, n) * n * n
        for b in offs:
            i01 = i0 + np.mod(cell[:, 1] + b, n) * n
            for e in offs:
                mark[i01 + np.mod(cell[:, 2] + e, n)] = True
    del h
    return int(mark.sum())


def algorithmic_bytes(stage, order, U):
    """Algorithmic HBM bytes of one launch of `stage` for this workload.

    gather      : positions (24 B) + u and grad u in FP32 (16 B * C) per particle,
                  plus every distinct coefficient touched once (C * 4 B per point)
    fft_axis0   : read the complex128 spectrum, write the complex64 work array
    fft_axis1   : read and write the complex64 work array
    fft_c2r     : read the work array, write the ghost-padded FP32 grid
    """
    n, C = N_GRID, NCOMP
    half = n * n * (n // 2 + 1) * C
    padded = (n + order - 1) ** 3 * C
    if stage == "gather":
        return P * (24 + 16 * C) + U * C * 4
    if stage == "fft_axis0":
        return half * (16 + 8)
    if stage == "fft_axis1":
        return half * 16
    if stage == "fft_c2r":
        return half * 8 + padded * 4
    return None


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_256cube_x3_f32_orders4_6_1e6.md")
KERNEL_SOURCES = {"gather": ["eval.hip", "gather.hpp", "common.hpp"], "fft": ["fft.hip", "common.hpp"]}


def measured_traffic(key):
    """HBM bytes per launch of stage `key` from the committed counter summary.

    The summary records FETCH_SIZE + WRITE_SIZE (scaled by a plain copy of
    known size) with a hash of the kernel's sources; the figure is returned
    only while the sources still hash the same, else None.
    """
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    line = next((ln for ln in text.splitlines() if ln.startswith("traffic-json:")), None)
    if line is None:
        return None
    table = json.loads(line.split(":", 1)[1])
    ent = table.get(key) or table.get(key.split("@N")[0])
    if ent is None:
        return None
    kind = "gather" if key.startswith("gather") else "fft"
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1201_4060_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return ent["traffic_bytes"] if h.hexdigest()[:16] == ent["src"] else None


def cpu_baseline(uhat, pos, sample):
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
    ap.add_argument("--form", choices=("plain", "copy"), default="plain",
                    help="plain: the interpolation workload (default); copy: 1 GiB device copy "
                         "used to calibrate HBM byte counters")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=100000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sort-tile", type=int, default=None)
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
    import synth
    import paper_1201_4060_amd as bsi
    from paper_1201_4060_amd import _bsi

    assert torch.cuda.is_available(), "bench.py needs a GPU"
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

    def step():
        for o in ORDERS:
            fields[o].set_spectrum(uhat)
            fields[o].eval(pos, cfg=cfg, out=outs[o])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for o in ORDERS:
        _bsi.bsi_ctx_reset_timing(ctxs[o].handle)
        _bsi.bsi_ctx_set_timing(ctxs[o].handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = len(ORDERS) * P / ((t1 - t0) / args.steps)

    stages = {}
    for o in ORDERS:
        for st in STAGES:
            ms, cnt = _bsi.bsi_ctx_read_timing(ctxs[o].handle, st)
            if cnt:
                stages[f"{st}@N{o}"] = {"avg_us": 1000.0 * ms / cnt, "launches": cnt,
                                        "total_ms": ms}
    for o in ORDERS:
        _bsi.bsi_ctx_set_timing(ctxs[o].handle, False)
    stage_ms_per_step = sum(v["total_ms"] for v in stages.values()) / args.steps
    eprint(f"{ms_per_step:.3f} ms/step wall, {stage_ms_per_step:.3f} ms/step in library kernels")
    for k, v in sorted(stages.items(), key=lambda kv: -kv[1]["total_ms"]):
        eprint(f"  {k:20s} {v['avg_us']:9.1f} us x {v['launches']}")

    # dominant kernel (largest share of the step among the kernels with an
    # algorithmic byte count: gather and FFT passes) and its roofline
    dom_key = max((k for k in stages if algorithmic_bytes(k.split("@N")[0], 4, 0) is not None),
                  key=lambda k: stages[k]["total_ms"])
    dom_stage, dom_order = dom_key.split("@N")
    dom_order = int(dom_order)
    U = distinct_stencil_points(pos_np, N_GRID, dom_order) if dom_stage == "gather" else 0
    alg = algorithmic_bytes(dom_stage, dom_order, U)
    avg_s = stages[dom_key]["avg_us"] * 1e-6
    achieved = alg / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom_key),
                "kernel": dom_key, "algorithmic_bytes": alg, "avg_us": round(stages[dom_key]["avg_us"], 2)}
    # the particle gather's own roofline beside it (the spec kernel)
    gather_rl = {}
    for o in ORDERS:
        k = f"gather@N{o}"
        if k in stages:
            Uo = distinct_stencil_points(pos_np, N_GRID, o)
            b = algorithmic_bytes("gather", o, Uo)
            a = b / (stages[k]["avg_us"] * 1e-6) / 1e9
            gather_rl[k] = {"achieved_GBs": round(a, 1), "frac": round(a / HBM_PEAK_GBS, 4),
                            "algorithmic_bytes": b, "distinct_points": Uo,
                            "avg_us": round(stages[k]["avg_us"], 2),
                            "points_per_s": round(P / (stages[k]["avg_us"] * 1e-6), 1)}

    cpu = None
    if not args.no_cpu_baseline:
        eprint("timing the CPU oracle on a sample ...")
        cpu = cpu_baseline(uhat_np, pos_np, args.cpu_sample)

    for o in ORDERS:
        fields[o].close()
        ctxs[o].close()

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256^3 x3 divergence-free Kolmogorov field, FP32 grid, orders 4 and 6, "
                               "1e6 uniform particles; step = prefilter + eval per order",
                   "n": N_GRID, "ncomp": NCOMP, "orders": list(ORDERS), "particles": P,
                   "grid_dtype": "f32", "spectrum_dtype": "c128", "parallelism": "single GPU"},
        "roofline": roofline,
        "gather_roofline": gather_rl,
        "stages_us": {k: round(v["avg_us"], 2) for k, v in stages.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
