"""MI355X (gfx950) D-SKI: Gaussian-process regression with derivatives.

The product is ``libdski.so`` (HIP kernels behind the C ABI in
``include/dski.h``); ``paper_1810_12283_amd.dski`` is its ctypes binding.
"""
from .dski import (DSKIError, DskipPlan, MarginalLikelihood, Mlp, Plan, Precond, lanczos_quad_log, lib, rademacher,  # noqa: F401
                   version)
