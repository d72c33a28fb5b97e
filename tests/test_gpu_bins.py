"""The evaluation's Morton binning (a counting sort of the particles by tile),
read back through bsi_debug_bins.

What is unique is compared exactly: every bucket's count and first binned slot
(the exclusive prefix sum of the counts) against a host counting sort of the
oracle's cells, and every binned position, bit for bit, against the position
of the particle its slot names.  What is not unique, the order of the particles
inside a bucket, is checked for validity: the slots hold a permutation of the
particles and every particle sits inside its own bucket's range of slots.
"""
import math

import numpy as np
import pytest

import synth
from gpu_common import log, dev, host, edge_positions

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1201_4060_amd import Context
    c = Context(0)
    yield c
    c.close()


def morton3(a, b, c, bits):
    """Interleave the bits of the tile coordinates, axis 0 highest of each triple."""
    k = np.zeros(a.shape, dtype=np.int64)
    for i in range(bits):
        k |= ((a >> i) & 1) << (3 * i + 2)
        k |= ((b >> i) & 1) << (3 * i + 1)
        k |= ((c >> i) & 1) << (3 * i)
    return k


def expected_bins(pos, shape, tile):
    from oracle import cells
    cell, _, fin = cells(pos, shape)
    bits = max(math.ceil(math.log2(-(-n // tile))) if n > tile else 0 for n in shape)
    nb = (1 << (3 * bits)) + 1
    key = morton3(cell[:, 0] // tile, cell[:, 1] // tile, cell[:, 2] // tile, bits)
    key = np.where(fin, key, nb - 1)
    hist = np.bincount(key, minlength=nb)
    offs = np.concatenate([[0], np.cumsum(hist)[:-1]])
    return key, hist, offs


def check_bins(f, pos, shape, tile):
    P = pos.shape[0]
    hist, offs, perm, ps = f.debug_bins(dev(pos), tile)
    hist, offs, perm, ps = host(hist), host(offs), host(perm).astype(np.int64), host(ps)
    key, h, o = expected_bins(pos, shape, tile)
    assert hist.shape == h.shape, (hist.shape, h.shape)
    assert np.array_equal(hist.astype(np.int64), h), "bucket counts"
    assert np.array_equal(offs.astype(np.int64), o), "bucket first slots"
    assert np.array_equal(np.sort(perm), np.arange(P)), "slots are not a permutation"
    slot_bucket = np.repeat(np.arange(h.shape[0]), h)
    assert np.array_equal(key[perm], slot_bucket), "a particle outside its bucket's slots"
    assert np.array_equal(ps.view(np.uint64), pos[perm].view(np.uint64)), "binned positions"
    log(f"  bins {shape} tile {tile}: P={P}, {h.shape[0]} buckets, "
        f"{int((h > 0).sum())} non-empty, largest {int(h.max())}")


@pytest.mark.parametrize("tile", [1, 4, 8, 16])
def test_bins_small_grid(ctx, tile):
    from paper_1201_4060_amd import Field, BSI_F32
    pos = np.concatenate([synth.uniform_positions(20011, seed=60 + tile), edge_positions(),
                          np.array([[np.nan, 1.0, 2.0], [np.inf, 0.0, 0.0], [1.7e308, 0.0, 0.0]])])
    with Field(ctx, 64, 3, 4, BSI_F32) as f:
        check_bins(f, pos, (64, 64, 64), tile)


def test_bins_noncubic_and_ragged(ctx):
    # tile edges that do not divide the grid, axes of different lengths
    from paper_1201_4060_amd import Field, BSI_F32
    shape = (48, 96, 36)
    pos = synth.uniform_positions(30001, seed=61)
    with Field(ctx, shape, 1, 6, BSI_F32) as f:
        for tile in (5, 8, 12):
            check_bins(f, pos, shape, tile)


def test_bins_crowded(ctx):
    # 6e4 particles on one point among clustered ones: one bucket far above
    # the per-chunk size of the grouping, plus non-finite particles
    from paper_1201_4060_amd import Field, BSI_F32
    pos = np.concatenate([synth.clustered_positions(20000, 5, 8000, 0.05, seed=62),
                          np.tile([[1.0, 2.0, 3.0]], (60000, 1)),
                          np.full((7, 3), np.nan)])
    pos = pos[np.random.default_rng(63).permutation(pos.shape[0])]
    with Field(ctx, 128, 3, 4, BSI_F32) as f:
        check_bins(f, np.ascontiguousarray(pos), (128, 128, 128), 8)


def test_bins_empty_and_invalid(ctx):
    import torch
    from paper_1201_4060_amd import Field, BSI_F32, BsiError
    with Field(ctx, 32, 1, 4, BSI_F32) as f:
        hist, offs, perm, ps = f.debug_bins(torch.empty((0, 3), dtype=torch.float64, device="cuda"), 8)
        assert hist.shape[0] == 65 and int(hist.abs().sum()) == 0 and int(offs.abs().sum()) == 0
        assert perm.shape[0] == 0
        with pytest.raises(BsiError):
            f.debug_bins(dev(synth.uniform_positions(10, seed=1)), 0)
    with Field(ctx, 512, 1, 4, BSI_F32) as f:
        with pytest.raises(BsiError):   # 512 / 256 = 2: tile 1 would exceed the bucket table limit
            f.debug_bins(dev(synth.uniform_positions(10, seed=1)), 1)


@pytest.mark.parametrize("case", ["256cube_1e6_uniform", "512cube_1e7_clustered"])
def test_bins_full_size(ctx, case):
    # the binning of the benchmark's workloads, in the tile the evaluation uses there
    from paper_1201_4060_amd import Field, BSI_F32
    if case == "256cube_1e6_uniform":
        n, pos = 256, synth.uniform_positions(1_000_000, seed=101)
    else:
        n, pos = 512, synth.clustered_positions(5_000_000, 100, 50_000, 0.1, seed=102)
    log(f"bins full size {case}")
    with Field(ctx, n, 3, 6, BSI_F32) as f:
        check_bins(f, pos, (n, n, n), 8)
