"""Conventional GPW exchange on the device (AO-RI-K, Alg. 1; MO-RI-K, Alg. 2)
against the oracle's plain loops, and the occ-RI-K identities of Sec. II.D
between the device's conventional and occ-RI-K results."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle import collocation, conventional, occrik
import paper_2207_09028_amd as pkg
from paper_2207_09028_amd import OccrikError
from paper_2207_09028_amd.plan import Plan, PlanSpec

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu_required():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _case(grid, nocc, counts, kmesh=(2, 1, 2), kernel=W.KERNEL_COULOMB, omega=0.0, seed=23):
    prob = W.small_problem(kmesh=kmesh, grid=grid, nocc=nocc, counts=counts, kernel=kernel, omega=omega, seed=seed)
    C = W.random_coefficients(prob)
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
    return prob, C, chi


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# grids: odd sizes (run-time FFT sizes, generic pass 3) and a compiled cubic size;
# N_ao = 22 and 28 leave partial groups of output AOs (8 per pass group, 16 per contraction)
@pytest.mark.parametrize("algo", ["mo", "ao"])
@pytest.mark.parametrize("grid,nocc,counts,mode", [((12, 10, 9), 3, (2, 1, 1), "fftfreq"),
                                                   ((12, 10, 9), 2, (2, 2, 1), "symmetric"),
                                                   ((24, 24, 24), 4, (2, 1, 1), "symmetric")])
def test_conventional_k_matches_oracle_fp64(algo, grid, nocc, counts, mode):
    prob, C, chi = _case(grid, nocc, counts)
    ref_fn = conventional.mo_k if algo == "mo" else conventional.ao_k
    Kref = ref_fn(prob, C, chi, nyquist=mode)
    plan = Plan(PlanSpec.from_problem(prob, nyquist=1 if mode == "symmetric" else 0))
    out = plan.conventional_k(torch.from_numpy(C).to("cuda"), algo=algo)
    torch.cuda.synchronize()
    K = out["K"].cpu().numpy()
    assert _rel(K, Kref) < 1e-10
    e_ref = np.real(np.einsum("kai,kab,kbi->", C.conj(), Kref, C)) / (2 * prob.nk)
    assert abs(float(out["Ex"][0]) - e_ref) < 1e-10 * abs(e_ref)


@pytest.mark.parametrize("kernel,omega", [(W.KERNEL_ERF_LR, 0.4), (W.KERNEL_TRUNC_COULOMB, 0.0)])
def test_conventional_mo_k_other_kernels(kernel, omega):
    prob, C, chi = _case((12, 10, 9), 3, (2, 1, 1), kernel=kernel, omega=omega)
    Kref = conventional.mo_k(prob, C, chi)
    plan = Plan(PlanSpec.from_problem(prob, nyquist=0))
    K = plan.conventional_k(torch.from_numpy(C).to("cuda"), algo="mo")["K"].cpu().numpy()
    assert _rel(K, Kref) < 1e-10


@pytest.mark.parametrize("precision", [pkg.PREC_FP64, pkg.PREC_FP32_SPLIT])
def test_conventional_and_occrik_agree_on_the_occupied_space(precision):
    """K C = K_{mu j}, C^H K C = K_ij and one E_x for AO-RI-K, MO-RI-K and occ-RI-K
    (Sec. II.D), all three from the device in one precision mode."""
    prob, C, _ = _case((24, 24, 24), 4, (2, 1, 1), kmesh=(2, 2, 1))
    plan = Plan(PlanSpec.from_problem(prob, nyquist=1, precision=precision))
    Ct = torch.from_numpy(C).to("cuda")
    occ = plan.build(Ct)
    Kmi, Ex = occ["Kmi"].cpu().numpy(), float(occ["Ex"][0])
    tol_rel = 1e-10 if precision == pkg.PREC_FP64 else 1e-5
    for algo in ("mo", "ao"):
        out = plan.conventional_k(Ct, algo=algo)
        torch.cuda.synchronize()
        K = out["K"].cpu().numpy()
        assert _rel(np.einsum("kab,kbi->kai", K, C), Kmi) < tol_rel
        assert np.max(np.abs(K - K.conj().transpose(0, 2, 1))) < tol_rel * np.max(np.abs(K))
        tol_e = 1e-10 * abs(Ex) if precision == pkg.PREC_FP64 else 1e-6
        assert abs(float(out["Ex"][0]) - Ex) < tol_e


def test_conventional_fp32_split_meets_the_accuracy_gate():
    prob, C, chi = _case((24, 24, 24), 4, (2, 1, 1))
    Kref = conventional.mo_k(prob, C, chi, nyquist="symmetric")
    e_ref = np.real(np.einsum("kai,kab,kbi->", C.conj(), Kref, C)) / (2 * prob.nk)
    plan = Plan(PlanSpec.from_problem(prob, nyquist=1, precision=pkg.PREC_FP32_SPLIT))
    Ct = torch.from_numpy(C).to("cuda")
    for algo in ("mo", "ao"):
        out = plan.conventional_k(Ct, algo=algo)
        torch.cuda.synchronize()
        assert np.max(np.abs(out["K"].cpu().numpy() - Kref)) <= 1e-5
        assert abs(float(out["Ex"][0]) - e_ref) <= 1e-6


def test_conventional_uses_the_occupied_columns_of_an_extended_plan():
    prob, C, chi = _case((12, 10, 9), 5, (2, 1, 1))
    Ct = torch.from_numpy(C).to("cuda")
    ext = Plan(PlanSpec.from_problem(prob, nocc=3, nvir=2, nyquist=0))
    occ = Plan(PlanSpec.from_problem(prob, nocc=3, nyquist=0))
    Ke = ext.conventional_k(Ct, algo="mo")["K"].cpu().numpy()
    Ko = occ.conventional_k(Ct[:, :, :3].contiguous(), algo="mo")["K"].cpu().numpy()
    assert _rel(Ke, Ko) < 1e-14
    Kref = conventional.mo_k(prob, C[:, :, :3], chi)
    assert _rel(Ke, Kref) < 1e-10


def test_conventional_repeated_calls_and_algorithm_switch_are_stable():
    """Workspaces grow from MO-RI-K (N_occ summed) to AO-RI-K (N_ao summed) and are
    reused; results do not depend on the call history."""
    prob, C, _ = _case((12, 10, 9), 3, (2, 1, 1))
    Ct = torch.from_numpy(C).to("cuda")
    plan = Plan(PlanSpec.from_problem(prob))
    k1 = plan.conventional_k(Ct, algo="mo")["K"].cpu().numpy()
    a1 = plan.conventional_k(Ct, algo="ao")["K"].cpu().numpy()
    k2 = plan.conventional_k(Ct, algo="mo")["K"].cpu().numpy()
    fresh = Plan(PlanSpec.from_problem(prob))
    a2 = fresh.conventional_k(Ct, algo="ao")["K"].cpu().numpy()
    assert np.array_equal(k1, k2)
    assert np.array_equal(a1, a2)


def test_conventional_rejects_direct_plans_and_unknown_algorithms():
    prob, C, _ = _case((12, 10, 9), 3, (2, 1, 1))
    Ct = torch.from_numpy(C).to("cuda")
    direct = Plan(PlanSpec.from_problem(prob, flags=pkg.FLAG_DIRECT))
    with pytest.raises(OccrikError) as e:
        direct.conventional_k(Ct, algo="mo")
    assert e.value.status == 2
    plan = Plan(PlanSpec.from_problem(prob))
    with pytest.raises(ValueError):
        plan.conventional_k(Ct, algo="xx")
    # the library's own check of the algorithm code and of the required K
    K = torch.empty((prob.nk, plan.nao, plan.nao), dtype=torch.complex128, device="cuda")
    lib = pkg.load()
    c_ptr, k_ptr = ctypes.c_void_p(Ct.data_ptr()), ctypes.c_void_p(K.data_ptr())
    assert lib.occrik_conventional_k(plan._h, 3, c_ptr, k_ptr, None) == 1
    assert lib.occrik_conventional_k(plan._h, pkg.ALGO_MO_RI_K, c_ptr, None, None) == 1
