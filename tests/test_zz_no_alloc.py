"""occrik_build_static, the build for callers that cannot allocate device memory,
against occrik_build on the same plans: two calls in a row, the second with a smaller
input (the staging array keeps the first call's contents), and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
import paper_2207_09028_amd as pkg
from paper_2207_09028_amd import OccrikError, _lib
from paper_2207_09028_amd.plan import Plan, PlanSpec

pytestmark = pytest.mark.gpu


def _static(plan, C):
    """occrik_build_static through the C ABI."""
    lib = _lib.load()
    C = np.ascontiguousarray(C, dtype=np.complex128)
    K = np.full((plan.nk, plan.nao, plan.nao), np.nan, np.complex128)
    Kmi = np.full((plan.nk, plan.nao, plan.ncol), np.nan, np.complex128)
    Ex = ctypes.c_double(np.nan)
    plan._sync_stream()
    st = lib.occrik_build_static(plan._h, ctypes.c_void_p(C.ctypes.data), ctypes.c_void_p(K.ctypes.data),
                                 ctypes.c_void_p(Kmi.ctypes.data), ctypes.byref(Ex))
    _lib.check(st, plan._h)
    return dict(K=K, Kmi=Kmi, Ex=Ex.value)


def test_static_build_equals_build_on_two_calls_the_second_smaller():
    assert torch.cuda.is_available()
    # first call: 125 k-points x 190 AOs, whose K~ (72 MB) is staged in two groups of k-points
    big = W.small_problem(kmesh=(5, 5, 5), grid=(12, 12, 12), nocc=4, counts=(20, 15, 5), amin=0.5, seed=21)
    small = W.small_problem(kmesh=(2, 1, 2), grid=(12, 10, 9), nocc=3, seed=22)
    assert big.nao == 190 and big.nk * big.nao ** 2 * 16 > 64 << 20
    for prob, prec in ((big, pkg.PREC_FP64), (small, pkg.PREC_FP32_SPLIT)):
        C = W.random_coefficients(prob)
        plan = Plan(PlanSpec.from_problem(prob, precision=prec))
        ref = plan.build_host(C)                    # occrik_build
        out = _static(plan, C)
        assert np.array_equal(out["K"], ref["K"]), prob.name
        assert np.array_equal(out["Kmi"], ref["Kmi"]), prob.name
        assert out["Ex"] == ref["Ex"], prob.name
        plan.close()


def test_static_build_rejects_plans_beyond_its_staging_array():
    # 512 k-points x 350 AOs x 16 columns: C and K_{mu j} need 2 x 45.9 MB of staging
    prob = W.Problem("wide", W.diamond_cell(), W.even_tempered_basis(2, [20, 15, 10, 5], 0.5, 50.0),
                     (8, 8, 8), (4, 4, 4), 16)
    plan = Plan(PlanSpec.from_problem(prob))
    C = np.ones((plan.nk, plan.nao, plan.ncol), np.complex128)
    with pytest.raises(OccrikError) as e:
        _static(plan, C)
    assert e.value.status == 1 and "staging" in str(e.value)
    plan.close()
