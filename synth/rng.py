"""Counter-based SplitMix64.

SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) advances a 64-bit state by the odd constant
GAMMA and returns a bijective mix of the new state.  Because the k-th output
depends only on (initial state + k*GAMMA), any output can be computed directly
from its counter, which is what lets every workload element be drawn
independently and reproducibly at any size.

All arithmetic here is on numpy uint64 arrays, which wrap modulo 2**64.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_S30 = np.uint64(30)
_S27 = np.uint64(27)
_S31 = np.uint64(31)
_S11 = np.uint64(11)
_INV53 = 1.0 / 9007199254740992.0  # 2**-53


def splitmix64_mix(z):
    """The SplitMix64 output mix of a (already advanced) state z (uint64 array)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _S30)) * _M1
        z = (z ^ (z >> _S27)) * _M2
    return z ^ (z >> _S31)


def _stream_base(seed, stream):
    """Initial state of the (seed, stream) sequence."""
    with np.errstate(over="ignore"):
        s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GAMMA
        s = splitmix64_mix(np.array([s ^ np.uint64(stream & 0xFFFFFFFFFFFFFFFF)],
                                    dtype=np.uint64))[0]
    return s


def keyed_u64(seed, stream, counter):
    """counter-th output (0-based) of the SplitMix64 sequence of (seed, stream).

    counter: integer array (any shape, values >= 0).  Returns uint64 array.
    """
    base = _stream_base(seed, stream)
    c = np.asarray(counter).astype(np.uint64)
    with np.errstate(over="ignore"):
        state = base + (c + np.uint64(1)) * GAMMA
    return splitmix64_mix(state)


def keyed_uniform(seed, stream, counter):
    """Uniform doubles in [0, 1) from the top 53 bits of keyed_u64."""
    return (keyed_u64(seed, stream, counter) >> _S11).astype(np.float64) * _INV53
