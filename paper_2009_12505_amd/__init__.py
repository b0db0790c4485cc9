"""MI355X (gfx950) build of the screened periodic Hartree-Fock exchange matrix
under the localized resolution of identity (Lin, Ren & He).

Python is only the marshalling layer over the C ABI of ``libhfx.so``
(``include/hfx.h``): every step of the build runs in the library's HIP
kernels.  PyTorch provides device memory and streams.

    plan = Plan(cells, C, V, D_pattern, thresholds)
    sigma = plan.build(D)          # list of float64 CUDA tensors, one per cell
    e_x = plan.energy(D, sigma)    # list of floats
"""
from ._abi import (HfxError, PREC_BF16X3, PREC_FP32, PREC_FP64, PREC_TIERED, SCHED_EXACT, SCHED_KMEANS, SCHED_LPT, SCHED_MLP, SCHED_NORM, SCHED_PLAN,
                   SCREEN_ALL, SCREEN_CS1, SCREEN_CS2, SCREEN_CS3, SCREEN_CS_ERI, SCREEN_PRE, lib)
from .plan import Plan

__all__ = ["Plan", "HfxError", "lib", "PREC_FP64", "PREC_FP32", "PREC_TIERED", "PREC_BF16X3", "SCHED_PLAN",
           "SCHED_LPT", "SCHED_MLP", "SCHED_EXACT", "SCHED_NORM", "SCHED_KMEANS", "SCREEN_ALL", "SCREEN_PRE", "SCREEN_CS_ERI", "SCREEN_CS1", "SCREEN_CS2",
           "SCREEN_CS3"]
