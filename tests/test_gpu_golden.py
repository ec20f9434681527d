"""GPU parity at the full workload sizes against stored oracle results.

The ``.npz`` files under ``tests/golden`` are written by
``tests/golden/make_golden.py``, which calls only the FP64 oracle and the
seeded workload generators.  The GPU runs here use the same plan settings the
benchmark times (symmetric Nyquist, automatic k batching, register-resident
transforms on these cubic grids).

Bars: FP64 1e-10 relative (max-norm over each array, relative energies);
FP32 (plain or with split-bf16 contractions) |dE_x| <= 1e-6 Eh and max |dK~| <= 1e-5.
"""
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import occrik
import paper_2207_09028_amd as pkg
from paper_2207_09028_amd.plan import Plan, PlanSpec

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL64 = 1e-10
EX_TOL_REDUCED = 1e-6
K_TOL_REDUCED = 1e-5


@pytest.fixture(autouse=True)
def _gpu_required():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def golden(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return np.load(path)


def gpu_build(prob, C, precision):
    plan = Plan(PlanSpec.from_problem(prob, nyquist=pkg.NYQUIST_SYMMETRIC, precision=precision))
    out = plan.build(torch.from_numpy(C).to("cuda"))
    return plan, {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("name", ["prec", "diff"])
def test_full_workload_fp64(name):
    g = golden(name)
    prob = W.make_problem(name)
    C = W.random_coefficients(prob)
    plan, out = gpu_build(prob, C, pkg.PREC_FP64)
    assert rel(out["Kmi"], g["Kmi"]) < TOL64
    assert rel(out["K"][:2], g["K_sample"]) < TOL64
    assert abs(out["Ex"][0] - float(g["Ex"])) < TOL64 * abs(float(g["Ex"]))
    Kij = occrik.occupied_block(C, out["Kmi"])
    assert rel(Kij, g["Kij"]) < TOL64
    if "dEx_domega" in g.files:
        _, dw = plan.grad(want_C=False, want_omega=True)
        assert abs(dw - float(g["dEx_domega"])) < TOL64 * abs(float(g["dEx_domega"]))


@pytest.mark.parametrize("precision", [pkg.PREC_FP32_SPLIT, pkg.PREC_FP32])
@pytest.mark.parametrize("name", ["prec", "diff"])
def test_full_workload_reduced_precision(name, precision):
    """Complex64 transforms with split-bf16 (or plain FP32) contractions and FP64
    reductions, against the stored FP64 oracle values at the reduced-precision bars."""
    g = golden(name)
    prob = W.make_problem(name)
    C = W.random_coefficients(prob)
    plan, out = gpu_build(prob, C, precision)
    assert abs(out["Ex"][0] - float(g["Ex"])) <= EX_TOL_REDUCED
    assert np.max(np.abs(out["K"][:2] - g["K_sample"])) <= K_TOL_REDUCED
    assert np.max(np.abs(out["Kmi"] - g["Kmi"])) <= K_TOL_REDUCED
    if "dEx_domega" in g.files:
        # the adjoint of the reduced-precision forward (FP64 reductions): dE_x/dC =
        # (2/N_k) K_{mu j} (from eq. exxao) at the K bar, dE_x/domega within 1e-5 relative
        gC, dw = plan.grad(want_C=True, want_omega=True)
        ref = occrik.energy_gradient_C(g["Kmi"], prob.nk)
        assert np.max(np.abs(gC.cpu().numpy() - ref)) <= (2.0 / prob.nk) * K_TOL_REDUCED
        assert abs(dw - float(g["dEx_domega"])) <= 1e-5 * abs(float(g["dEx_domega"]))


@pytest.mark.parametrize("precision", [pkg.PREC_FP64, pkg.PREC_FP32_SPLIT, pkg.PREC_FP32])
def test_paper_workload_sampled_kpoints(precision):
    """6x6x6 k, 350 AO, 8 occupied, 48^3: the whole build on the GPU, checked on the
    output k-points the oracle computed exactly (each sums over all 216 k')."""
    g = golden("paper")
    prob = W.make_problem("paper")
    C = W.random_coefficients(prob)
    _, out = gpu_build(prob, C, precision)
    ks = [int(k) for k in g["k"]]
    Kmi = out["Kmi"][ks]
    K = out["K"][ks][:, g["K_rows"]]
    terms = occrik.exchange_energy_terms(occrik.occupied_block(C[ks], Kmi), prob.nk)
    if precision == pkg.PREC_FP64:
        assert rel(Kmi, g["Kmi"]) < TOL64
        assert rel(K, g["K"]) < TOL64
        assert rel(terms, g["ex_terms"]) < TOL64
    else:
        assert np.max(np.abs(K - g["K"])) <= K_TOL_REDUCED
        # per-k energy terms enter E_x one by one; each within the energy bar over N_k
        assert np.max(np.abs(terms - g["ex_terms"])) <= EX_TOL_REDUCED / prob.nk
