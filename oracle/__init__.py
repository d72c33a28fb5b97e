"""FP64 CPU oracle for B-spline (and comparison-method) interpolation of spectral fields.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP library
never links, imports or executes anything here, and this package never touches
the HIP library: the two share no code (the seeded input generator in
``synth/`` is the only thing both consume).

It computes, plainly and slowly, what the method of van Hinsberg, ten Thije
Boonkkamp, Toschi and Clercx, "On the efficiency and accuracy of interpolation
methods for spectral codes" (SIAM J. Sci. Comput. 2012) defines:

* ``bspline``  -- the interpolation matrix M_(N) (Section 7, general formula)
                  and M^(l) = M D^l (Section 2);
* ``symbol``   -- the Fourier-space prefilter constants c(k), both the
                  straightforward 1/F_D[B_D] and the L2-optimal choice
                  (Section 7);
* ``prefilter``-- c(kx)c(ky)c(kz) times the spectrum, then one inverse real
                  FFT (Section 7, 3D multiplication and method statement);
* ``evaluate`` -- stencil selection (Section 5, nearest-grid-point rule) and
                  the direct triple sum of weights times coefficients
                  (Section 3, n-mode products), with first derivatives,
                  and with second derivatives (M^(2) = M D^2, Section 2);
* ``methods``  -- the comparison methods' matrices: Lagrange through the N
                  nearest points (linear for N = 2) and Hermite (Sections 2, 8);
                  ``evaluate(..., basis="lagrange")`` runs them on grid values
                  (prefilter variant NONE, c = 1);
* ``hermite``  -- cubic Hermite in 3D: the 8 derivative fields per component
                  from the spectrum and the plain 4^3-entry tensor sum
                  (Sections 2, 3, 6);
* ``theory``   -- per-mode relative L2 errors (Sections 5, 6, 8) of every
                  method: the curves of Figs 3 and 4, used as pins.

Every function is pinned by ``tests/test_oracle_*.py`` against values fixed by
the paper and by mathematics (printed matrices, closed forms, brute force on
tiny grids, polynomial reproduction, convergence order).
"""
from .bspline import (bspline_matrix, derivative_matrix, matrix_f64,
                      derivative_matrix_f64)
from .symbol import sinc_power_sum, prefilter_constants, INTERP, L2OPT, NONE
from .prefilter import prefilter
from .evaluate import (cells, weights, weights2, evaluate, evaluate_hessian, inv_spacing, TWO_PI,
                       HESS_PAIRS)
from .methods import lagrange_matrix, hermite_matrix
from . import theory, hermite

__all__ = [
    "bspline_matrix", "derivative_matrix", "matrix_f64", "derivative_matrix_f64",
    "sinc_power_sum", "prefilter_constants", "INTERP", "L2OPT", "NONE",
    "lagrange_matrix", "hermite_matrix", "hermite",
    "prefilter", "cells", "weights", "evaluate", "inv_spacing", "TWO_PI",
    "theory",
]
