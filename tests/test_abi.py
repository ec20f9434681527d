"""CPU checks of the C ABI: the library loads, exports every declared symbol, and
rejects bad inputs before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2207_09028_amd as pkg
from paper_2207_09028_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "occrik.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(occrik_[a-z_]+)\s*\(", text)))


def test_header_declares_the_expected_entry_points():
    names = declared_functions()
    for n in ["occrik_plan_create", "occrik_build", "occrik_build_device", "occrik_build_batch", "occrik_grad",
              "occrik_plan_destroy", "occrik_last_error_k", "occrik_status_string"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pkg.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    # the binding declares the same set
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_status_strings_and_supported_sizes():
    lib = pkg.load()
    for code, name in _lib.STATUS_NAMES.items():
        assert lib.occrik_status_string(code).decode() == name
    for n in [1, 2, 3, 5, 9, 12, 24, 30, 36, 40, 48, 64]:
        assert lib.occrik_grid_size_supported(n) == 1
    for n in [0, 7, 11, 13, 49, 65, 96, -4]:
        assert lib.occrik_grid_size_supported(n) == 0


def _create(**override):
    lib = pkg.load()
    lat = (ctypes.c_double * 9)(*np.eye(3).reshape(9) * 5.0)
    atoms = np.zeros(3)
    cell = _lib.Cell(lat, 1, atoms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    sa = np.zeros(2, np.int32)
    sl = np.array([0, override.pop("l", 1)], np.int32)
    se = np.array([1.0, override.pop("alpha", 0.5)])
    basis = _lib.Basis(2, sa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                       sl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                       se.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    p = dict(kmesh=(1, 1, 1), grid=(8, 8, 8), nocc=1, kernel=0, omega=0.0, nyquist=1, precision=0,
             lattice_tol=1e-12, kbatch=0, flags=0, mem_budget=0, nvir=0, contract_chunks=0)
    p.update(override)
    params = _lib.Params((ctypes.c_int32 * 3)(*p["kmesh"]), (ctypes.c_int32 * 3)(*p["grid"]), p["nocc"],
                         p["kernel"], p["omega"], p["nyquist"], p["precision"], p["lattice_tol"], p["kbatch"],
                         p["flags"], p["mem_budget"], p["nvir"], p["contract_chunks"])
    h = _lib.PlanP()
    st = lib.occrik_plan_create(ctypes.byref(cell), ctypes.byref(basis), ctypes.byref(params), 0, None,
                                ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("override,status", [
    (dict(grid=(8, 7, 8)), 2),          # 7 is not 2^a 3^b 5^c
    (dict(grid=(8, 8, 96)), 2),         # beyond the largest supported extent
    (dict(l=4), 2),                     # g functions are not supported
    (dict(nocc=0), 1),
    (dict(contract_chunks=-1), 1),
    (dict(contract_chunks=65), 1),
    (dict(nocc=17), 1),
    (dict(nvir=-1), 1),
    (dict(nocc=10, nvir=7), 1),         # nocc + nvir above 16
    (dict(kernel=1, omega=0.0), 1),     # range-separated kernel without omega
    (dict(kernel=7), 1),
    (dict(precision=5), 1),
    (dict(nyquist=3), 1),
    (dict(lattice_tol=0.0), 1),
    (dict(kmesh=(0, 1, 1)), 1),
    (dict(flags=16), 1),                # undefined flag bit
    (dict(flags=3), 1),                 # LDS_FFT and REG_FFT_ALL together
    (dict(alpha=-1.0), 1),
])
def test_plan_create_rejects_bad_inputs_before_any_device_work(override, status):
    st, h = _create(**override)
    assert st == status
    assert not h.value
    assert pkg.load().occrik_last_error_message().decode()


def test_null_arguments_are_rejected():
    lib = pkg.load()
    assert lib.occrik_plan_create(None, None, None, 0, None, None) == 1
    assert lib.occrik_build(None, None, None, None, None) == 1
    assert lib.occrik_build_device(None, None, None, None, None) == 1
    assert lib.occrik_grad(None, 1.0, None, None) == 1
    assert lib.occrik_plan_autotune(None, None, None) == 1
    assert lib.occrik_conventional_k(None, 2, None, None, None) == 1
    assert lib.occrik_last_error_k(None) == -1
    lib.occrik_plan_destroy(None)


def test_profile_traffic_reads_as_unmeasured_after_a_change(tmp_path):
    """The committed HBM-counter summaries count only while the hashed sources are unchanged:
    the hash covers every listed file, in order."""
    import hashlib
    from paper_2207_09028_amd.profiling import sources_sha256
    (tmp_path / "a").write_bytes(b"kernel")
    (tmp_path / "b").write_bytes(b"launch")
    h = sources_sha256("a,b", str(tmp_path))
    assert h == hashlib.sha256(b"kernellaunch").hexdigest()
    assert sources_sha256("b,a", str(tmp_path)) != h
    (tmp_path / "b").write_bytes(b"launch2")
    assert sources_sha256("a,b", str(tmp_path)) != h


def test_hbm_probe_rejects_bad_arguments_before_any_device_work():
    lib = pkg.load()
    buf = ctypes.c_void_p(4096)          # never dereferenced: every case fails validation first
    ms = ctypes.c_double()
    for kind, width, every, nbytes, reps in [(4, 16, 0, 1024, 1), (-1, 16, 0, 1024, 1), (0, 12, 0, 1024, 1),
                                            (1, 16, 0, 0, 1), (1, 16, 0, 1000, 1), (1, 16, 0, 1024, 0),
                                            (3, 16, 0, 1024, 1)]:
        assert lib.occrik_hbm_probe(kind, width, 0, every, buf, buf, nbytes, reps, None, ctypes.byref(ms)) == 1
    assert lib.occrik_hbm_probe(0, 16, 0, 0, buf, buf, 1024, 1, None, None) == 1
