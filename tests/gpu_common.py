"""Helpers shared by the GPU parity tests (imported only by tests marked gpu)."""
import sys

import numpy as np

TOL_F64 = 1e-12   # FP64 grid and arithmetic (a proposed bound; the paper fixes none)
TOL_F32 = 1e-5    # FP32 coefficients and arithmetic


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_err(got, want):
    """max |got - want| / max |want| over each quantity (last axis flattened away).

    got/want: [P][...]; returns the per-quantity maxima as a flat array.
    """
    g = np.asarray(got, dtype=np.float64).reshape(got.shape[0], -1)
    w = np.asarray(want, dtype=np.float64).reshape(want.shape[0], -1)
    num = np.max(np.abs(g - w), axis=0)
    den = np.max(np.abs(w), axis=0)
    return num / np.where(den > 0, den, 1.0)


def bf16_round(a):
    """Round float64 -> float32 -> bfloat16 (nearest, ties to even) -> float64.

    The test-side model of BF16 storage (IEEE definition of the rounding).
    """
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def edge_positions(L=2 * np.pi):
    return np.array([
        [0.0, 0.0, 0.0],
        [L, L, L],
        [np.nextafter(L, 0.0), np.nextafter(0.0, 1.0), -0.0],
        [np.nextafter(0.0, -1.0), -1e-300, -L],
        [-3.7, 13.1, -8.25],
        [2 * L, 3 * L, -5 * L],
        [1e15, -1e15, 1e17],
        [1e300, -1e300, 7.0],
        [L / 2, L / 4, L / 8],
    ])
