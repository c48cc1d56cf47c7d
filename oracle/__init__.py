"""FP64 CPU oracle for the local ETKF analysis/forecast step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import this package.  The product path
(the HIP library and its Python binding) never imports, links or calls it,
and this package imports nothing from the product path.

It is a plain, slow, step-by-step restatement of what the paper's method
computes, in float64 NumPy (LAPACK ``eigh`` for the eigenproblem):

* ``letkf``   ensemble mean/perturbations, slope synthesis, per-domain
              analysis, merge, AR forecast (paper Sec. 2.1-2.3; the ETKF
              transform of the cited refs [8]-[10], [14], symmetric square
              root per ref [9]).
* ``philox``  Philox4x32-10 counter-based generator (Salmon et al., SC'11)
              and Box-Muller normals, used for the forecast model noise.

Parity pins (tests marked ``not gpu``) tie every function to something other
than itself: closed forms, the Kalman-filter identity, library routines and
brute force; see the test files for the list.
"""
from .letkf import (analysis, domain_analysis, ensemble_mean_perturbations, forecast,
                    frame_step, slope_synthesis)
from .philox import forecast_normals, philox4x32_10, box_muller

__all__ = ["analysis", "domain_analysis", "ensemble_mean_perturbations", "forecast",
           "frame_step", "slope_synthesis", "forecast_normals", "philox4x32_10", "box_muller"]
