"""Python face of the occ-RI-K library: the same entry points as ``include/occrik.h``.

PyTorch supplies device memory and the current HIP stream; every step of a
build runs in the library's HIP kernels.  Arrays follow the C layouts:

    C    [N_k, N_ao, nocc + nvir]  complex128  occupied coefficients, then nvir conduction bands
    K    [N_k, N_ao, N_ao]  complex128  assembled exchange matrix K~
    Kmi  [N_k, N_ao, nocc + nvir]  complex128  K_{mu j}
    Ex   scalar float64                  exchange energy per cell and spin
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import ALGO_AO_RI_K, ALGO_MO_RI_K, check


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class PlanSpec:
    lattice: np.ndarray            # (3, 3) bohr, rows a_1..a_3
    atoms_frac: np.ndarray         # (natm, 3)
    shell_atom: np.ndarray         # (nshell,)
    shell_l: np.ndarray            # (nshell,)
    shell_exp: np.ndarray          # (nshell,)
    kmesh: tuple
    grid: tuple
    nocc: int
    kernel: int = _lib.KERNEL_COULOMB
    omega: float = 0.0
    nyquist: int = _lib.NYQUIST_SYMMETRIC
    precision: int = _lib.PREC_FP64
    lattice_tol: float = 1e-12
    kbatch: int = 0
    mem_budget: int = 0
    flags: int = 0
    nvir: int = 0
    contract_chunks: int = 0

    @classmethod
    def from_problem(cls, prob, **overrides):
        """From any object with cell/basis/kmesh/grid/nocc/kernel/omega/lattice_tol attributes."""
        kw = dict(lattice=np.asarray(prob.cell.lattice, dtype=np.float64),
                  atoms_frac=np.asarray(prob.cell.atoms_frac, dtype=np.float64),
                  shell_atom=np.asarray(prob.basis.shell_atom, dtype=np.int32),
                  shell_l=np.asarray(prob.basis.shell_l, dtype=np.int32),
                  shell_exp=np.asarray(prob.basis.shell_exp, dtype=np.float64),
                  kmesh=tuple(prob.kmesh), grid=tuple(prob.grid), nocc=int(prob.nocc),
                  kernel=int(prob.kernel), omega=float(prob.omega), lattice_tol=float(prob.lattice_tol))
        kw.update(overrides)
        return cls(**kw)


class Plan:
    """An occ-RI-K plan on one GPU (wraps occrik_plan_create / occrik_plan_destroy)."""

    def __init__(self, spec: PlanSpec, device=None):
        lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the occ-RI-K library needs a HIP device")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.spec = spec
        lat = np.ascontiguousarray(spec.lattice, dtype=np.float64).reshape(9)
        self._atoms = np.ascontiguousarray(spec.atoms_frac, dtype=np.float64).reshape(-1)
        self._sa = np.ascontiguousarray(spec.shell_atom, dtype=np.int32)
        self._sl = np.ascontiguousarray(spec.shell_l, dtype=np.int32)
        self._se = np.ascontiguousarray(spec.shell_exp, dtype=np.float64)
        cell = _lib.Cell((ctypes.c_double * 9)(*lat), len(self._atoms) // 3,
                         self._atoms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        basis = _lib.Basis(len(self._sl), self._sa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           self._sl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           self._se.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        params = _lib.Params((ctypes.c_int32 * 3)(*spec.kmesh), (ctypes.c_int32 * 3)(*spec.grid), int(spec.nocc),
                             int(spec.kernel), float(spec.omega), int(spec.nyquist), int(spec.precision),
                             float(spec.lattice_tol), int(spec.kbatch), int(spec.flags), int(spec.mem_budget),
                             int(spec.nvir), int(spec.contract_chunks))
        handle = _lib.PlanP()
        with torch.cuda.device(self.device):
            st = lib.occrik_plan_create(ctypes.byref(cell), ctypes.byref(basis), ctypes.byref(params),
                                        self.device.index, _stream_handle(self.device), ctypes.byref(handle))
        check(st)
        self._h = handle
        self._lib = lib
        self.info = self.query()
        self.nk, self.nao, self.nocc, self.ng = self.info.nk, self.info.nao, self.info.nocc, self.info.ng
        self.nvir = self.info.nvir
        self.ncol = self.nocc + self.nvir        # columns of C, K_{mu j}, psi~ and W~
        # bumped by every call that replaces the state occrik_grad reads (the last
        # build's K_{mu j} and orbitals, and omega), so that an adjoint can tell whether
        # the plan still holds the build it belongs to
        self.generation = 0

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.occrik_plan_destroy(self._h)
            self._h = _lib.PlanP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- queries --------------------------------------------------------------
    def query(self):
        info = _lib.PlanInfo()
        check(self._lib.occrik_plan_query(self._h, ctypes.byref(info)))
        return info

    def _sync_stream(self):
        check(self._lib.occrik_set_stream(self._h, _stream_handle(self.device)))

    def set_omega(self, omega: float):
        check(self._lib.occrik_set_omega(self._h, float(omega)))
        self.generation += 1

    # -- builds ---------------------------------------------------------------
    def _check_C(self, C):
        if not isinstance(C, torch.Tensor) or C.dtype != torch.complex128 or C.device != self.device:
            raise TypeError("C must be a complex128 tensor on the plan's device")
        if tuple(C.shape) != (self.nk, self.nao, self.ncol) or not C.is_contiguous():
            raise ValueError(f"C must be contiguous with shape {(self.nk, self.nao, self.ncol)}")

    def build_device(self, C, K=None, Kmi=None, Ex=None):
        """occrik_build_device on caller tensors (asynchronous on the current stream)."""
        self._check_C(C)
        for t, shape in ((K, (self.nk, self.nao, self.nao)), (Kmi, (self.nk, self.nao, self.ncol))):
            if t is not None and (t.dtype != torch.complex128 or tuple(t.shape) != shape or not t.is_contiguous()
                                  or t.device != self.device):
                raise ValueError(f"output must be contiguous complex128 {shape} on the plan's device")
        if Ex is not None and (Ex.dtype != torch.float64 or Ex.numel() != 1 or Ex.device != self.device):
            raise ValueError("Ex must be one float64 on the plan's device")
        self._sync_stream()
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        self.generation += 1
        check(self._lib.occrik_build_device(self._h, ptr(C), ptr(K), ptr(Kmi), ptr(Ex)), self._h)

    def status(self):
        check(self._lib.occrik_plan_status(self._h), self._h)

    def build(self, C, want_K=True, want_Kmi=True):
        """Build and return dict(K, Kmi, Ex) as device tensors; raises on a deferred device error."""
        dev = self.device
        K = torch.empty((self.nk, self.nao, self.nao), dtype=torch.complex128, device=dev) if want_K else None
        Kmi = torch.empty((self.nk, self.nao, self.ncol), dtype=torch.complex128, device=dev) if want_Kmi else None
        Ex = torch.empty((1,), dtype=torch.float64, device=dev)
        self.build_device(C, K, Kmi, Ex)
        self.status()
        return dict(K=K, Kmi=Kmi, Ex=Ex)

    def autotune(self, C):
        """occrik_plan_autotune: time builds of C over the open settings (k batch, pair
        transform form, contraction chunks) and keep the fastest; returns a dict of the
        choice and the timings.  Synchronous."""
        self._check_C(C)
        self._sync_stream()
        ti = _lib.TuneInfo()
        self.generation += 1
        check(self._lib.occrik_plan_autotune(self._h, ctypes.c_void_p(C.data_ptr()), ctypes.byref(ti)), self._h)
        self.info = self.query()
        return dict(kbatch=ti.kbatch, reg_fft=ti.reg_fft, contract_chunks=ti.contract_chunks, builds=ti.builds,
                    ms_initial=ti.ms_initial, ms_best=ti.ms_best)

    def conventional_k(self, C, algo="mo", K=None, Ex=None):
        """occrik_conventional_k: the full AO x AO exchange matrix by MO-RI-K (Alg. 2,
        ``algo="mo"``) or AO-RI-K (Alg. 1, ``algo="ao"``) on this plan's grid and kernel.
        Returns dict(K, Ex) as device tensors; asynchronous on the current stream."""
        code = {"ao": ALGO_AO_RI_K, "mo": ALGO_MO_RI_K}.get(algo)
        if code is None:
            raise ValueError("algo must be 'ao' or 'mo'")
        self._check_C(C)
        dev = self.device
        shape = (self.nk, self.nao, self.nao)
        if K is None:
            K = torch.empty(shape, dtype=torch.complex128, device=dev)
        elif K.dtype != torch.complex128 or tuple(K.shape) != shape or not K.is_contiguous() or K.device != dev:
            raise ValueError(f"K must be contiguous complex128 {shape} on the plan's device")
        if Ex is None:
            Ex = torch.empty((1,), dtype=torch.float64, device=dev)
        elif Ex.dtype != torch.float64 or Ex.numel() != 1 or Ex.device != dev:
            raise ValueError("Ex must be one float64 on the plan's device")
        self._sync_stream()
        check(self._lib.occrik_conventional_k(self._h, code, ctypes.c_void_p(C.data_ptr()),
                                              ctypes.c_void_p(K.data_ptr()), ctypes.c_void_p(Ex.data_ptr())), self._h)
        return dict(K=K, Ex=Ex)

    def build_host(self, C: np.ndarray, want_K=True, want_Kmi=True):
        """occrik_build: synchronous, host arrays in and out."""
        C = np.ascontiguousarray(C, dtype=np.complex128)
        if C.shape != (self.nk, self.nao, self.ncol):
            raise ValueError("bad C shape")
        K = np.empty((self.nk, self.nao, self.nao), np.complex128) if want_K else None
        Kmi = np.empty((self.nk, self.nao, self.ncol), np.complex128) if want_Kmi else None
        Ex = ctypes.c_double(0.0)
        p = lambda a: ctypes.c_void_p(a.ctypes.data) if a is not None else None
        self._sync_stream()
        self.generation += 1
        check(self._lib.occrik_build(self._h, p(C), p(K), p(Kmi), ctypes.byref(Ex)), self._h)
        return dict(K=K, Kmi=Kmi, Ex=Ex.value)

    def build_host_static(self, C: np.ndarray, want_K=True, want_Kmi=True):
        """occrik_build_static: occrik_build staged through the library's static device
        array (no device allocation per call); synchronous, host arrays in and out."""
        C = np.ascontiguousarray(C, dtype=np.complex128)
        if C.shape != (self.nk, self.nao, self.ncol):
            raise ValueError("bad C shape")
        K = np.empty((self.nk, self.nao, self.nao), np.complex128) if want_K else None
        Kmi = np.empty((self.nk, self.nao, self.ncol), np.complex128) if want_Kmi else None
        Ex = ctypes.c_double(0.0)
        p = lambda a: ctypes.c_void_p(a.ctypes.data) if a is not None else None
        self._sync_stream()
        self.generation += 1
        check(self._lib.occrik_build_static(self._h, p(C), p(K), p(Kmi), ctypes.byref(Ex)), self._h)
        return dict(K=K, Kmi=Kmi, Ex=Ex.value)

    def grad(self, gEx=1.0, want_C=True, want_omega=False):
        """occrik_grad after a build: dL/dC (device tensor) and dL/domega (float)."""
        g = torch.empty((self.nk, self.nao, self.ncol), dtype=torch.complex128, device=self.device) if want_C else None
        dw = ctypes.c_double(0.0)
        self._sync_stream()
        check(self._lib.occrik_grad(self._h, float(gEx), ctypes.c_void_p(g.data_ptr()) if g is not None else None,
                                    ctypes.byref(dw) if want_omega else None))
        return g, (dw.value if want_omega else None)

    # -- diagnostics and profiling -----------------------------------------------
    def intermediate(self, which: str):
        idx = {"chi": 0, "psi": 1, "W": 2}[which]
        rows = self.nao if idx == 0 else self.ncol
        out = torch.empty((self.nk, rows, self.ng), dtype=torch.complex128, device=self.device)
        self._sync_stream()
        check(self._lib.occrik_copy_intermediate(self._h, idx, ctypes.c_void_p(out.data_ptr()),
                                                 out.numel() * 16))
        return out

    def set_profiling(self, level: int):
        check(self._lib.occrik_set_profiling(self._h, int(level)))

    def profile(self, reset=True):
        p = _lib.Profile()
        check(self._lib.occrik_get_profile(self._h, ctypes.byref(p), 1 if reset else 0))
        out = {}
        for f, _ in _lib.Profile._fields_:
            v = getattr(p, f)
            out[f] = list(v) if hasattr(v, "__len__") else v
        return out


def build_batch(plans, Cs, Ks=None, Kmis=None, Exs=None):
    """occrik_build_batch over plans that share the current stream."""
    lib = _lib.load()
    n = len(plans)
    for p in plans:
        p._sync_stream()
    arr = lambda xs: (ctypes.c_void_p * n)(*[ctypes.c_void_p(x.data_ptr()) if x is not None else None for x in xs])
    hp = (_lib.PlanP * n)(*[p._h for p in plans])
    none = [None] * n
    for p in plans:
        p.generation += 1
    st = lib.occrik_build_batch(n, hp, arr(Cs), arr(Ks or none), arr(Kmis or none), arr(Exs or none))
    check(st)


class BatchGraph:
    """occrik_batch_create / occrik_batch_launch / occrik_batch_destroy: a ragged batch
    recorded once as a HIP graph and replayed with one launch.  The plans must share a
    non-default stream (the current one when recorded); the plans and tensors passed
    here must stay alive while the object is used.  ``fused=True`` records it with
    occrik_batch_create_fused (fused pair-pass rounds for plans that share a kernel
    form); ``self.fused`` is the number of plans that run in such rounds."""

    def __init__(self, plans, Cs, Ks=None, Kmis=None, Exs=None, fused=False):
        lib = _lib.load()
        n = len(plans)
        for p in plans:
            p._sync_stream()
        arr = lambda xs: (ctypes.c_void_p * n)(*[ctypes.c_void_p(x.data_ptr()) if x is not None else None for x in xs])
        hp = (_lib.PlanP * n)(*[p._h for p in plans])
        none = [None] * n
        self._keep = (plans, Cs, Ks, Kmis, Exs)
        self._h = ctypes.c_void_p()
        for p in plans:
            p.generation += 1
        create = lib.occrik_batch_create_fused if fused else lib.occrik_batch_create
        check(create(n, hp, arr(Cs), arr(Ks or none), arr(Kmis or none), arr(Exs or none), ctypes.byref(self._h)))
        self._lib = lib
        nf = ctypes.c_int32()
        check(lib.occrik_batch_fused(self._h, ctypes.byref(nf)))
        self.fused = nf.value          # plans whose pair passes run in fused rounds

    def launch(self):
        for p in self._keep[0]:
            p.generation += 1
        check(self._lib.occrik_batch_launch(self._h))

    def close(self):
        if self._h:
            self._lib.occrik_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def grid_size_supported(n: int) -> bool:
    return bool(_lib.load().occrik_grid_size_supported(int(n)))
