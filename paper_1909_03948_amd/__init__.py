"""MI355X-native Hessian actions for Bayesian inversion of the Poisson
log-coefficient problem (Villa, Petra & Ghattas, hIPPYlib Part I).

The compute path is libhinv.so (HIP, gfx950) behind the C ABI of
include/hinv.h; ``paper_1909_03948_amd.hinv`` is its thin ctypes binding.
"""
from .hinv import (Context, HinvError, Problem, load, HESS_FULL, HESS_MISFIT, HESS_GN_FULL,
                   HESS_GN_MISFIT, PREC_FP64, PREC_FP32_IR, TPROD_FP64, TPROD_BF16)

__all__ = ["Context", "HinvError", "Problem", "load", "HESS_FULL", "HESS_MISFIT",
           "HESS_GN_FULL", "HESS_GN_MISFIT", "PREC_FP64", "PREC_FP32_IR", "TPROD_FP64",
           "TPROD_BF16"]
