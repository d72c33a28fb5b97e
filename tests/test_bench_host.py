"""Host logic of bench.py (no GPU): algorithmic byte counts, the distinct
stencil-point count, the comment-insensitive kernel-source hash that guards the
recorded HBM traffic, and the refusal of more than one GPU."""
import itertools
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_gather_bytes_formula():
    # positions (24 B) + u and grad u (4 C values of out_bytes) per particle,
    # plus C coefficients of coef_bytes per distinct grid point
    assert bench.gather_bytes(10, 3, 100, 4) == 10 * (24 + 12 * 4) + 100 * 3 * 4
    assert bench.gather_bytes(1, 1, 64, 8, out_bytes=8) == 24 + 4 * 8 + 64 * 8


def test_fft_bytes_formula():
    n, C = 256, 3
    half = n * n * (n // 2 + 1) * C
    assert bench.fft_bytes("fft_axis0", n, C, 6) == half * (16 + 8)
    assert bench.fft_bytes("fft_axis1", n, C, 6) == half * 16
    assert bench.fft_bytes("fft_c2r", n, C, 6) == half * 8 + (n + 5) ** 3 * C * 4
    assert bench.fft_bytes("gather", n, C, 6) is None


def _brute_distinct(pos, n, order):
    cell = np.floor(pos * (n / (2 * np.pi))).astype(np.int64) % n
    offs = [o - order // 2 + 1 for o in range(order)]
    pts = set()
    for c in cell:
        for a, b, e in itertools.product(offs, offs, offs):
            pts.add(((c[0] + a) % n, (c[1] + b) % n, (c[2] + e) % n))
    return len(pts)


@pytest.mark.parametrize("n,order,P", [(8, 4, 1), (8, 4, 3), (16, 6, 40), (12, 4, 200)])
def test_distinct_stencil_points_brute_force(n, order, P):
    import torch
    pos = np.random.default_rng(n * 100 + P).uniform(0, 2 * np.pi, size=(P, 3))
    got = bench.distinct_stencil_points(torch.from_numpy(pos), n, order)
    assert got == _brute_distinct(pos, n, order)


def test_distinct_stencil_points_limits():
    import torch
    one = torch.tensor([[1.0, 2.0, 3.0]], dtype=torch.float64)
    assert bench.distinct_stencil_points(one, 16, 6) == 6 ** 3
    dense = torch.from_numpy(np.random.default_rng(1).uniform(0, 2 * np.pi, size=(4000, 3)))
    assert bench.distinct_stencil_points(dense, 8, 4) == 8 ** 3


def _fake_sources(tmp_path, body):
    d = tmp_path / "paper_1201_4060_amd" / "csrc"
    d.mkdir(parents=True, exist_ok=True)
    for f in ("eval.hip", "gather.hpp", "common.hpp", "fft.hip"):
        (d / f).write_text(body)


def test_kernel_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _fake_sources(tmp_path, "int f(int x) {\n  return x + 1;\n}\n")
    h0 = bench.kernel_source_hash("gather")
    _fake_sources(tmp_path, "// a comment\nint f(int x) { /* block\n comment */\n    return x + 1;  // tail\n}\n")
    assert bench.kernel_source_hash("gather") == h0
    _fake_sources(tmp_path, "int f(int x) {\n  return x + 2;\n}\n")
    assert bench.kernel_source_hash("gather") != h0


def test_measured_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _fake_sources(tmp_path, "int g() { return 7; }\n")
    h = bench.kernel_source_hash("gather")
    t = tmp_path / "traffic.md"
    t.write_text('text\ntraffic-json: {"gather@N6": {"traffic_bytes": 123, "src": "%s"}, '
                 '"fft_c2r": {"traffic_bytes": 9, "src": "0000"}}\n' % h)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(t))
    assert bench.measured_traffic("gather@N6") == 123
    assert bench.measured_traffic("fft_c2r@N6") is None      # recorded for other sources
    assert bench.measured_traffic("gather@N4") is None       # not recorded
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("gather@N6") is None


def test_roofline_entry():
    e = bench.roofline_entry("gather@N6", 8e9, 1000.0, traffic=10)
    assert e["achieved"] == pytest.approx(8000.0) and e["frac"] == pytest.approx(1.0)
    assert e["peak"] == 8000.0 and e["unit"] == "GB/s" and e["bound"] == "hbm" and e["traffic"] == 10


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_gather_fma_count():
    # 6N^3 + 15N^2 + 12N for three components: 672 (N = 4), 1908 (N = 6)
    assert bench.gather_fma(4, 3) == 672 and bench.gather_fma(6, 3) == 1908
    assert bench.gather_fma(4, 1) == 2 * 64 + 9 * 16 + 16
    assert bench.FMA_PEAK_PER_S == pytest.approx(39.32e12, rel=1e-3)


def test_hessian_fma_count():
    # 3 FMAs per coefficient (w, w', w'' along axis 2), 6 per row, 10 per plane
    assert bench.hessian_fma(6, 3) == 3 * 3 * 216 + 6 * 3 * 36 + 10 * 3 * 6 == 2772
    assert bench.hessian_fma(4, 1) == 3 * 64 + 6 * 16 + 40
