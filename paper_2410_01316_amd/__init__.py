"""MI355X-native QMC-slicing fast kernel summation.

    plan = Plan(xi, kernel="gauss", n_ft=128, scale=sigma, R=R, n_max=N, m_max=M)
    s = plan(x, w, y)                      # torch float32 tensors on the GPU

The computation lives in libfastsum.so (HIP kernels for gfx950 behind the C
ABI of include/fastsum.h); this package only marshals arguments.
"""
from ._lib import FastSumError, load as load_library, LIB_PATH
from .api import (Plan, FastSum, Batch, kernel_sum, distance_qmc, host_tables, choose_nft,
                  bound)
from .flow import MMDFlow

__all__ = ["Plan", "FastSum", "Batch", "MMDFlow", "kernel_sum", "distance_qmc", "FastSumError",
           "host_tables", "choose_nft", "bound", "load_library", "LIB_PATH"]
