"""MI355X (gfx950) implementation of the cyclic-to-cyclic multidimensional FFT
with a single all-to-all (Koopman & Bisseling, arXiv 2203.11795, Algorithm 2.3).

The transform runs in the HIP kernels of ``libfftu.so`` (C ABI in
``include/fftu.h``); :mod:`.fftu` is its Python binding.
"""
from .fftu import (C64, C128, FORWARD, INVERSE, NOALLOC_MAX_BYTES, BatchPlan, ConvolutionPlan, FftuError, Graph, Plan,
                   R2RPlan, RealPlan, check, describe, fill_uniform, get_tuning, load_library, pointwise_mul, set_tuning)

__all__ = ["Plan", "RealPlan", "R2RPlan", "BatchPlan", "ConvolutionPlan", "Graph", "FftuError", "check", "describe", "fill_uniform",
           "pointwise_mul", "load_library",
           "set_tuning", "get_tuning", "FORWARD", "INVERSE", "C64", "C128", "NOALLOC_MAX_BYTES"]
