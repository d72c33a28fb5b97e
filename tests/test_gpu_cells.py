"""GPU cell index and offset: bit-exact against the oracle (Section 5 stencil rule)."""
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


@pytest.mark.parametrize("n", [8, 32, 192, 256, 1024])
def test_cells_bit_exact(ctx, n):
    from paper_1201_4060_amd import Field, BSI_F32
    from oracle import cells
    log(f"cells n={n}")
    rng = np.random.default_rng(n)
    pos = np.concatenate([
        synth.uniform_positions(5003, seed=n),
        rng.uniform(-100.0, 100.0, size=(2000, 3)),
        # exact grid nodes and their neighbours
        (np.arange(50)[:, None] * (2 * np.pi / n)) * np.ones((1, 3)),
        np.nextafter((np.arange(50)[:, None] * (2 * np.pi / n)) * np.ones((1, 3)), -np.inf),
        edge_positions(),
    ])
    with Field(ctx, n, 1, 4, BSI_F32) as f:
        cell, t = f.debug_cells(dev(pos))
        cell, t = host(cell), host(t)
    ocell, ot, fin = cells(pos, (n, n, n))
    assert fin.all()
    assert np.array_equal(cell, ocell.astype(np.int32))
    assert np.array_equal(t.view(np.uint64), ot.view(np.uint64))


def test_cells_nonfinite(ctx):
    from paper_1201_4060_amd import Field, BSI_F32
    from oracle import cells
    pos = np.array([[np.nan, 0, 0], [0, np.inf, 0], [0, 0, -np.inf], [1.7e308, 0, 0], [1.0, 2.0, 3.0]])
    with Field(ctx, 32, 1, 4, BSI_F32) as f:
        cell, t = f.debug_cells(dev(pos))
        cell, t = host(cell), host(t)
    _, _, fin = cells(pos, (32, 32, 32))
    assert list(fin) == [False, False, False, False, True]
    assert (cell[:4] == -1).all() and np.isnan(t[:4]).all()
    assert (cell[4] >= 0).all()


def test_cells_empty(ctx):
    import torch
    from paper_1201_4060_amd import Field, BSI_F32
    with Field(ctx, 16, 1, 4, BSI_F32) as f:
        cell, t = f.debug_cells(torch.empty((0, 3), dtype=torch.float64, device="cuda"))
    assert cell.shape == (0, 3)
