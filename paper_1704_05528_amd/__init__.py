"""MI355X (gfx950) fast singular value thresholding with recycling rank-revealing randomized SVD.

Every step of the SVT / R4SVD iteration runs in the HIP kernels of libsvt.so
(csrc/); this package only marshals arguments across its C-ABI
(include/svt.h).  There is no CPU fallback: without the built library or
without a GPU the calls raise.
"""
from ._capi import (SVT_DTYPE_F32, SVT_DTYPE_F64, SVT_GRAD_DEVICE_POINTERS, SVT_GRAD_FROZEN_BASIS,
                    SVT_E_HIP, SVT_E_INVALID_ARG, SVT_E_LIMIT, SVT_E_NUMERIC, SVT_E_OOM, SVT_E_STATE,
                    SVT_F_ANNEALED, SVT_F_CONVERGED, SVT_F_EIG_INEXACT, SVT_F_EXHAUSTED, SVT_F_MAXIT,
                    SVT_F_RMAX_HIT, SVT_BF16, SVT_FP64, SVT_MIXED, SVT_MODE_R3SVD, SVT_MODE_R4SVD, SVT_MODE_RSVD, SVTError,
                    StepStats, default_params, lib_path, load, require_gpu)
from .svt import SVT, r4svd_step, svt_grad, svt_init, svt_iterate

__all__ = ["SVT", "svt_init", "r4svd_step", "svt_iterate", "svt_grad", "default_params", "StepStats", "SVTError",
           "load", "lib_path", "require_gpu", "SVT_FP64", "SVT_MIXED", "SVT_BF16", "SVT_MODE_R4SVD", "SVT_MODE_R3SVD",
           "SVT_MODE_RSVD", "SVT_DTYPE_F64", "SVT_DTYPE_F32", "SVT_GRAD_FROZEN_BASIS", "SVT_GRAD_DEVICE_POINTERS"]
