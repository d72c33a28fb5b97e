"""Seeded synthetic inputs shared by the GPU tests, the benchmark and the oracle tests.

This package draws random numbers and shapes them into workloads (Kolmogorov
spectra, particle clouds).  It holds none of the interpolation method's
arithmetic: no B-spline, no symbol, no transform, no stencil.  Both the HIP
path and the CPU oracle receive exactly the arrays produced here.
"""
from .rng import GAMMA, splitmix64_mix, keyed_u64, keyed_uniform
from .fields import kolmogorov_spectrum, spectrum_nonzero_count
from .particles import uniform_positions, clustered_positions

__all__ = [
    "GAMMA", "splitmix64_mix", "keyed_u64", "keyed_uniform",
    "kolmogorov_spectrum", "spectrum_nonzero_count",
    "uniform_positions", "clustered_positions",
]
