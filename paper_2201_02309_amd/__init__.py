"""MI355X (gfx950) pitch-by-pitch Katsevich helical FBP.

The compute path is the C-ABI shared library ``libkatsevich.so`` (hand-written HIP
kernels + float64 host plan) declared in ``include/katsevich.h``; this package holds
that library's sources (``csrc/``), its build step and a thin ctypes binding.
"""
from .katsevich import (Plan, KatsevichError, recon, recon_backward, filter_views,
                        backproject, backproject_batch, filtered_shape, KatsevichFn,
                        load_library, TABLES, sparse_upsample, max_value, add_noise, rmse_ssim,
                        rmse_ssim_noscratch)

__all__ = ["Plan", "KatsevichError", "recon", "recon_backward", "filter_views", "backproject",
           "backproject_batch", "filtered_shape", "KatsevichFn", "load_library", "TABLES",
           "sparse_upsample", "max_value", "add_noise", "rmse_ssim",
           "rmse_ssim_noscratch"]
