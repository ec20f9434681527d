"""occ-RI-K exact exchange for k-point GPW solids on MI355X (gfx950).

The compute path is the HIP library ``libocrik.so`` (C ABI in
``include/occrik.h``); this package only marshals arguments to it.  Importing
the package does not load the library; the first plan does, and raises if the
library is missing.
"""
from ._lib import (KERNEL_COULOMB, KERNEL_ERF_LR, KERNEL_ERFC_SR, KERNEL_TRUNC_COULOMB, KERNEL_TRUNC_ERF_LR, NYQUIST_FFTFREQ, NYQUIST_SYMMETRIC,
                   PREC_FP32, PREC_FP32_SPLIT, PREC_FP64, FLAG_LDS_FFT, FLAG_REG_FFT_ALL, FLAG_DIRECT, FLAG_MADELUNG, ALGO_AO_RI_K, ALGO_MO_RI_K,
                   OccrikError, LIB_PATH, load)

__all__ = ["Plan", "PlanSpec", "build_batch", "BatchGraph", "ExchangeEnergy", "exchange_energy", "load", "OccrikError",
           "KERNEL_COULOMB", "KERNEL_ERF_LR", "KERNEL_ERFC_SR", "KERNEL_TRUNC_COULOMB", "KERNEL_TRUNC_ERF_LR", "NYQUIST_FFTFREQ", "NYQUIST_SYMMETRIC",
           "PREC_FP64", "PREC_FP32", "PREC_FP32_SPLIT", "FLAG_LDS_FFT", "FLAG_REG_FFT_ALL", "FLAG_DIRECT", "FLAG_MADELUNG", "ALGO_AO_RI_K", "ALGO_MO_RI_K", "LIB_PATH"]


def __getattr__(name):
    if name in ("Plan", "PlanSpec", "build_batch", "BatchGraph", "grid_size_supported"):
        from . import plan
        return getattr(plan, name)
    if name in ("ExchangeEnergy", "exchange_energy"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
