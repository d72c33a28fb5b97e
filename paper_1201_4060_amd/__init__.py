"""B-spline interpolation of periodic spectral fields on MI355X (gfx950).

The method (van Hinsberg et al., "On the efficiency and accuracy of
interpolation methods for spectral codes"): a Fourier-space prefilter followed
by one inverse FFT gives the B-spline coefficient grid (Section 7); particles
are evaluated by a separable tensor-product contraction over their N^3 stencil
(Sections 2, 3, 5; Table 1).  Everything runs in the HIP library libbsi.so;
this package only marshals arguments to its C ABI (include/bsi.h).

torch is used for device memory and streams only.
"""
from . import _bsi
from ._bsi import (BsiError, BSI_F64, BSI_F32, BSI_BF16, BSI_PREFILTER_L2OPT,
                   BSI_PREFILTER_INTERP, BSI_PREFILTER_NONE, BSI_BASIS_BSPLINE, BSI_BASIS_LAGRANGE,
                   BSI_BASIS_HERMITE, EvalConfig)
from .api import Batch, Context, EvalPlan, Field, Server

__all__ = ["_bsi", "BsiError", "BSI_F64", "BSI_F32", "BSI_BF16", "BSI_PREFILTER_L2OPT",
           "BSI_PREFILTER_INTERP", "BSI_PREFILTER_NONE", "BSI_BASIS_BSPLINE", "BSI_BASIS_LAGRANGE",
           "BSI_BASIS_HERMITE", "EvalConfig", "Batch", "Context", "EvalPlan", "Field", "Server"]
