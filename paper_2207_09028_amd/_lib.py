"""ctypes declarations of the C ABI in ``include/occrik.h`` (argument marshalling only).

The shared library is loaded from the package directory.  There is no
fallback: if ``libocrik.so`` is missing or does not load, every entry point
raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libocrik.so")

OK = 0
STATUS_NAMES = {
    0: "OCCRIK_OK", 1: "OCCRIK_ERR_INVALID_ARG", 2: "OCCRIK_ERR_UNSUPPORTED", 3: "OCCRIK_ERR_OOM",
    4: "OCCRIK_ERR_NOT_PD", 5: "OCCRIK_ERR_NONFINITE", 6: "OCCRIK_ERR_DEVICE", 7: "OCCRIK_ERR_STATE",
}

KERNEL_COULOMB, KERNEL_ERF_LR, KERNEL_ERFC_SR, KERNEL_TRUNC_COULOMB, KERNEL_TRUNC_ERF_LR = 0, 1, 2, 3, 4
NYQUIST_FFTFREQ, NYQUIST_SYMMETRIC = 0, 1
PREC_FP64, PREC_FP32, PREC_FP32_SPLIT = 0, 1, 2
FLAG_LDS_FFT = 1
FLAG_REG_FFT_ALL = 2
FLAG_DIRECT = 4
FLAG_MADELUNG = 8
ALGO_AO_RI_K, ALGO_MO_RI_K = 1, 2

# every function the header declares, with (restype, argtypes)
c_int32 = ctypes.c_int32
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p


class Cell(ctypes.Structure):
    _fields_ = [("lattice", c_double * 9), ("natm", c_int32), ("atom_frac", ctypes.POINTER(c_double))]


class Basis(ctypes.Structure):
    _fields_ = [("nshell", c_int32), ("shell_atom", ctypes.POINTER(c_int32)),
                ("shell_l", ctypes.POINTER(c_int32)), ("shell_exp", ctypes.POINTER(c_double))]


class Params(ctypes.Structure):
    _fields_ = [("kmesh", c_int32 * 3), ("grid", c_int32 * 3), ("nocc", c_int32), ("kernel", c_int32),
                ("omega", c_double), ("nyquist", c_int32), ("precision", c_int32), ("lattice_tol", c_double),
                ("kbatch", c_int32), ("flags", c_int32), ("mem_budget", c_size_t), ("nvir", c_int32),
                ("contract_chunks", c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("nk", c_int32), ("nao", c_int32), ("nocc", c_int32), ("ng", c_int32),
                ("grid", c_int32 * 3), ("kmesh", c_int32 * 3),
                ("precision", c_int32), ("nyquist", c_int32), ("kernel", c_int32), ("kbatch", c_int32),
                ("omega", c_double), ("cell_volume", c_double),
                ("bytes_chi", c_size_t), ("bytes_workspace", c_size_t),
                ("pair_transforms", ctypes.c_int64), ("plan_seconds", c_double),
                ("integral_direct", c_int32), ("colloc_chunk", c_int32), ("reg_fft_passes", c_int32),
                ("nvir", c_int32), ("contract_chunks", c_int32), ("tuned", c_int32)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("kbatch", c_int32), ("reg_fft", c_int32), ("contract_chunks", c_int32), ("builds", c_int32),
                ("ms_initial", c_double), ("ms_best", c_double)]


class Profile(ctypes.Structure):
    _fields_ = [("ms_orbitals", c_double), ("ms_pairs", c_double), ("ms_contract", c_double),
                ("ms_assemble", c_double), ("launches_pairs", ctypes.c_int64), ("builds", ctypes.c_int64),
                ("ms_pass", c_double * 3), ("launches_pass", ctypes.c_int64 * 3), ("bytes_pass", c_double * 3)]


PlanP = c_void_p

SIGNATURES = {
    "occrik_plan_create": (c_int32, [ctypes.POINTER(Cell), ctypes.POINTER(Basis), ctypes.POINTER(Params),
                                     ctypes.c_int, c_void_p, ctypes.POINTER(PlanP)]),
    "occrik_plan_destroy": (None, [PlanP]),
    "occrik_plan_query": (c_int32, [PlanP, ctypes.POINTER(PlanInfo)]),
    "occrik_set_stream": (c_int32, [PlanP, c_void_p]),
    "occrik_set_omega": (c_int32, [PlanP, c_double]),
    "occrik_build": (c_int32, [PlanP, c_void_p, c_void_p, c_void_p, c_void_p]),
    "occrik_build_device": (c_int32, [PlanP, c_void_p, c_void_p, c_void_p, c_void_p]),
    "occrik_build_static": (c_int32, [PlanP, c_void_p, c_void_p, c_void_p, c_void_p]),
    "occrik_conventional_k": (c_int32, [PlanP, c_int32, c_void_p, c_void_p, c_void_p]),
    "occrik_plan_autotune": (c_int32, [PlanP, c_void_p, ctypes.POINTER(TuneInfo)]),
    "occrik_plan_status": (c_int32, [PlanP]),
    "occrik_last_error_k": (c_int32, [PlanP]),
    "occrik_grad": (c_int32, [PlanP, c_double, c_void_p, ctypes.POINTER(c_double)]),
    "occrik_build_batch": (c_int32, [c_int32, ctypes.POINTER(PlanP), ctypes.POINTER(c_void_p),
                                     ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p)]),
    "occrik_batch_create": (c_int32, [c_int32, ctypes.POINTER(PlanP), ctypes.POINTER(c_void_p),
                                      ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                      ctypes.POINTER(c_void_p)]),
    "occrik_batch_create_fused": (c_int32, [c_int32, ctypes.POINTER(PlanP), ctypes.POINTER(c_void_p),
                                      ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                      ctypes.POINTER(c_void_p)]),
    "occrik_batch_launch": (c_int32, [c_void_p]),
    "occrik_batch_destroy": (None, [c_void_p]),
    "occrik_batch_fused": (c_int32, [c_void_p, ctypes.POINTER(c_int32)]),
    "occrik_set_profiling": (c_int32, [PlanP, c_int32]),
    "occrik_get_profile": (c_int32, [PlanP, ctypes.POINTER(Profile), c_int32]),
    "occrik_copy_intermediate": (c_int32, [PlanP, c_int32, c_void_p, c_size_t]),
    "occrik_hbm_probe": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_size_t, c_int32,
                                   c_void_p, ctypes.POINTER(c_double)]),
    "occrik_status_string": (ctypes.c_char_p, [c_int32]),
    "occrik_last_error_message": (ctypes.c_char_p, []),
    "occrik_grid_size_supported": (c_int32, [c_int32]),
}

_lib = None


def load():
    """Load libocrik.so and declare every entry point; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"occ-RI-K HIP library not built: {LIB_PATH} is missing "
                           "(run python -m paper_2207_09028_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class OccrikError(RuntimeError):
    def __init__(self, status, message, k=None):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        self.k = k
        super().__init__(f"{self.name}: {message}" + (f" (k = {k})" if k is not None else ""))


def check(status, plan=None):
    if status == OK:
        return
    lib = load()
    msg = lib.occrik_last_error_message().decode(errors="replace")
    k = None
    if status == 4 and plan is not None:
        k = int(lib.occrik_last_error_k(plan))
    raise OccrikError(status, msg, k)
