"""Synthetic particle positions (FP64, [P][3]) on the periodic box [0, L)^3.

Streams of the counter-based generator used here (per seed):
  0..2   uniform coordinates of the uniform population (counter = particle)
  3..5   blob centres (counter = blob index)
  6..11  Box-Muller uniforms of the blob offsets, two streams per axis
  12     shuffle keys (counter = particle)
"""
import numpy as np

from .rng import keyed_uniform, keyed_u64

TWO_PI = 2.0 * np.pi


def uniform_positions(P, seed, L=TWO_PI):
    """P positions uniform in [0, L)^3."""
    idx = np.arange(P, dtype=np.int64)
    pos = np.empty((P, 3), dtype=np.float64)
    for d in range(3):
        pos[:, d] = keyed_uniform(seed, d, idx) * L
    return pos


def clustered_positions(P_uniform, n_blobs, per_blob, sigma, seed, L=TWO_PI,
                        shuffle=True):
    """Half-uniform / half-clustered cloud.

    P_uniform particles uniform in the box, then n_blobs Gaussian blobs of
    per_blob particles each (standard deviation sigma per axis, centres uniform),
    wrapped periodically into [0, L).  With shuffle=True the rows are put in a
    seeded random order, as a particle index from a simulation would be.
    """
    pos_u = uniform_positions(P_uniform, seed, L)
    nb = n_blobs * per_blob
    bidx = np.arange(n_blobs, dtype=np.int64)
    centres = np.stack([keyed_uniform(seed, 3 + d, bidx) * L for d in range(3)], axis=1)
    j = np.arange(nb, dtype=np.int64)
    pos_b = np.empty((nb, 3), dtype=np.float64)
    owner = j // per_blob
    for d in range(3):
        u1 = keyed_uniform(seed, 6 + 2 * d, j)
        u2 = keyed_uniform(seed, 7 + 2 * d, j)
        g = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(TWO_PI * u2)   # Box-Muller
        pos_b[:, d] = np.mod(centres[owner, d] + sigma * g, L)
    pos = np.concatenate([pos_u, pos_b], axis=0)
    if shuffle:
        keys = keyed_u64(seed, 12, np.arange(pos.shape[0], dtype=np.int64))
        pos = pos[np.argsort(keys, kind="stable")]
    return np.ascontiguousarray(pos)
