"""GPU parity of the HIP build against the FP64 oracle, stage by stage and end to end.

Inputs come from ``workloads`` (seeded); expected values from ``oracle`` only.
FP64 bar: 1e-10 relative (max-norm over each array).  Cell-periodic
intermediates of the library (chi~, psi~, W~ = e^{-ik.r} times the Bloch
quantity) are compared after applying that phase to the oracle's arrays.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import collocation, occrik
from oracle import lattice as olat
import paper_2207_09028_amd as pkg
from paper_2207_09028_amd.plan import Plan, PlanSpec

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


@pytest.fixture(autouse=True)
def _gpu_required():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def periodic_phase(prob):
    kc = olat.kpoints_cartesian(prob.cell.lattice, prob.kmesh)
    r = olat.grid_points(prob.cell.lattice, prob.grid)
    return np.exp(-1j * (kc @ r.T))               # [k, n]


_cache = {}


def oracle_result(prob, C, nyquist):
    key = (prob.name, prob.grid, prob.kmesh, prob.nocc, prob.kernel, prob.omega, nyquist, prob.seed)
    if key not in _cache:
        chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
        _cache[key] = occrik.build(prob, C, chi=chi, nyquist=nyquist, parseval=True,
                                   domega=prob.kernel != W.KERNEL_COULOMB)
    return _cache[key]


def run_gpu(prob, C, nyquist, precision=pkg.PREC_FP64, **kw):
    spec = PlanSpec.from_problem(prob, nyquist=1 if nyquist == "symmetric" else 0, precision=precision, **kw)
    plan = Plan(spec)
    Ct = torch.from_numpy(C).to("cuda")
    out = plan.build(Ct)
    return plan, {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


SMALL = [
    dict(kmesh=(2, 1, 3), grid=(12, 10, 9), nocc=3),
    dict(kmesh=(1, 1, 1), grid=(8, 9, 10), nocc=2),
    dict(kmesh=(3, 2, 1), grid=(15, 16, 6), nocc=4, counts=(2, 2, 1)),
]


@pytest.mark.parametrize("cfg", range(len(SMALL)))
@pytest.mark.parametrize("nyquist", ["symmetric", "fftfreq"])
def test_small_fp64_stagewise(cfg, nyquist):
    prob = W.small_problem(**SMALL[cfg])
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, nyquist)
    plan, out = run_gpu(prob, C, nyquist)
    ph = periodic_phase(prob)
    chi_ref = ref["chi"] * ph[:, None, :]
    psi_ref = ref["psi"] * ph[:, None, :]
    w_ref = ref["W"] * ph[:, None, :]
    errs = dict(
        chi=rel(plan.intermediate("chi").cpu().numpy(), chi_ref),
        psi=rel(plan.intermediate("psi").cpu().numpy(), psi_ref),
        W=rel(plan.intermediate("W").cpu().numpy(), w_ref),
        Kmi=rel(out["Kmi"], ref["Kmi"]),
        K=rel(out["K"], ref["K"]),
        Ex=abs(out["Ex"][0] - ref["Ex"]) / abs(ref["Ex"]),
    )
    print(cfg, nyquist, errs)
    for name, e in errs.items():
        assert e < TOL64, (name, e)


def test_tiny_fp64_end_to_end():
    prob = W.make_problem("tiny")
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, "symmetric")
    plan, out = run_gpu(prob, C, "symmetric")
    errs = dict(Kmi=rel(out["Kmi"], ref["Kmi"]), K=rel(out["K"], ref["K"]),
                Ex=abs(out["Ex"][0] - ref["Ex"]) / abs(ref["Ex"]))
    print("tiny", errs, out["Ex"][0], ref["Ex"])
    for name, e in errs.items():
        assert e < TOL64, (name, e)


@pytest.mark.parametrize("kernel,omega", [(W.KERNEL_ERF_LR, 0.3), (W.KERNEL_ERFC_SR, 0.45),
                                          (W.KERNEL_TRUNC_COULOMB, 0.0), (W.KERNEL_TRUNC_ERF_LR, 0.3)])
@pytest.mark.parametrize("mode", ["symmetric", "fftfreq"])
def test_other_kernels_fp64(kernel, omega, mode):
    """Range-separated and truncated Coulomb kernels (only the kernel multiply differs)."""
    prob = W.small_problem(kernel=kernel, omega=omega)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, mode)
    plan, out = run_gpu(prob, C, mode)
    assert rel(out["Kmi"], ref["Kmi"]) < TOL64
    assert rel(out["K"], ref["K"]) < TOL64
    assert abs(out["Ex"][0] - ref["Ex"]) < TOL64 * abs(ref["Ex"])


@pytest.mark.parametrize("kernel,omega", [(W.KERNEL_ERF_LR, 0.3), (W.KERNEL_ERFC_SR, 0.45),
                                          (W.KERNEL_TRUNC_COULOMB, 0.0), (W.KERNEL_TRUNC_ERF_LR, 0.3)])
def test_other_kernels_fp32_split_on_register_path(kernel, omega):
    """24^3 complex64 plans (the per-batch kernel-value table) with every kernel."""
    prob = W.small_problem(kmesh=(2, 1, 2), grid=(24, 24, 24), nocc=5, counts=(2, 2, 1), seed=33,
                           kernel=kernel, omega=omega)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, "symmetric")
    _, out = run_gpu(prob, C, "symmetric", precision=pkg.PREC_FP32_SPLIT)
    assert abs(out["Ex"][0] - ref["Ex"]) <= 1e-6
    assert np.max(np.abs(out["K"] - ref["K"])) <= 1e-5


@pytest.mark.parametrize("kernel,omega", [(W.KERNEL_TRUNC_COULOMB, 0.0), (W.KERNEL_TRUNC_ERF_LR, 0.7)])
def test_truncated_kernels_isolated_gaussian_on_gpu(kernel, omega):
    """The oracle's exact pins run through the library: one s-Gaussian per 8 bohr cell on a
    3x3x3 k-mesh gives E_x = -sqrt(mu/pi), mu = a for the cut-off 1/r and
    1/mu = 1/a + 1/w^2 for the cut-off erf(w r)/r."""
    alpha = 0.6
    mu = alpha if kernel == W.KERNEL_TRUNC_COULOMB else 1.0 / (1.0 / alpha + 1.0 / (omega * omega))
    cell = W.cubic_cell(8.0, [(0.5, 0.5, 0.5)])
    basis = W.Basis(np.zeros(1, np.int32), np.zeros(1, np.int32), np.array([alpha]))
    prob = W.Problem("sgauss", cell, basis, (3, 3, 3), (30, 30, 30), 1, seed=0, kernel=kernel, omega=omega)
    C = W.random_coefficients(prob)
    for precision, tol in ((pkg.PREC_FP64, 1e-11), (pkg.PREC_FP32_SPLIT, 1e-6)):
        _, out = run_gpu(prob, C, "symmetric", precision=precision)
        assert abs(out["Ex"][0] + np.sqrt(mu / np.pi)) < tol, precision


def test_batched_summed_kpoints_match_unbatched():
    """kbatch smaller than N_k (several FFT batches per output k, ragged last batch)."""
    prob = W.small_problem(kmesh=(3, 1, 2), grid=(10, 12, 8), nocc=3)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, "symmetric")
    _, out = run_gpu(prob, C, "symmetric", kbatch=4)
    assert rel(out["Kmi"], ref["Kmi"]) < TOL64
    assert abs(out["Ex"][0] - ref["Ex"]) < TOL64 * abs(ref["Ex"])


def test_fp64_builds_are_bitwise_reproducible():
    prob = W.small_problem()
    C = W.random_coefficients(prob)
    spec = PlanSpec.from_problem(prob)
    plan = Plan(spec)
    Ct = torch.from_numpy(C).to("cuda")
    a = plan.build(Ct)
    b = plan.build(Ct)
    assert torch.equal(a["K"], b["K"]) and torch.equal(a["Kmi"], b["Kmi"]) and torch.equal(a["Ex"], b["Ex"])


def test_host_entry_point_matches_device_entry_point():
    prob = W.small_problem()
    C = W.random_coefficients(prob)
    plan = Plan(PlanSpec.from_problem(prob))
    h = plan.build_host(C)
    d = plan.build(torch.from_numpy(C).to("cuda"))
    assert np.array_equal(h["K"], d["K"].cpu().numpy())
    assert h["Ex"] == float(d["Ex"][0])


def test_status_before_any_build_is_ok():
    prob = W.small_problem()
    plan = Plan(PlanSpec.from_problem(prob))
    plan.status()


@pytest.mark.parametrize("name", ["tiny", "tiny14"])
def test_specialised_grid_kernels_match_oracle_in_both_modes(name):
    """24^3 runs the compile-time-size pass kernels; both Nyquist modes (with and without pair reuse)."""
    prob = W.make_problem(name)
    C = W.random_coefficients(prob)
    for mode in ("fftfreq", "symmetric"):
        ref = oracle_result(prob, C, mode)
        _, out = run_gpu(prob, C, mode)
        assert rel(out["Kmi"], ref["Kmi"]) < TOL64
        assert rel(out["K"], ref["K"]) < TOL64
        assert abs(out["Ex"][0] - ref["Ex"]) < TOL64 * abs(ref["Ex"])


def test_pair_reuse_with_split_rows():
    """Symmetric mode with kbatch < N_k: rows of the upper triangle split across batches."""
    prob = W.small_problem(kmesh=(2, 2, 2), grid=(10, 9, 8), nocc=3)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, "symmetric")
    for kb in (1, 3, 5):
        _, out = run_gpu(prob, C, "symmetric", kbatch=kb)
        assert rel(out["Kmi"], ref["Kmi"]) < TOL64, kb
        assert abs(out["Ex"][0] - ref["Ex"]) < TOL64 * abs(ref["Ex"])


@pytest.mark.parametrize("flags", [0, pkg.FLAG_LDS_FFT])
@pytest.mark.parametrize("nocc,kbatch,mode", [(10, 0, "symmetric"), (3, 3, "symmetric"), (5, 2, "fftfreq"),
                                              (8, 0, "fftfreq"), (8, 3, "symmetric")])
def test_fused_pass3_variants_on_a_specialised_grid(nocc, kbatch, mode, flags):
    """24^3 grid: register and LDS transforms, 8 or 16 orbital lanes in pass 3, split rows, both Nyquist modes."""
    prob = W.small_problem(kmesh=(2, 1, 2), grid=(24, 24, 24), nocc=nocc, counts=(2, 2, 1), seed=21 + nocc)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, mode)
    _, out = run_gpu(prob, C, mode, kbatch=kbatch, flags=flags)
    assert rel(out["Kmi"], ref["Kmi"]) < TOL64
    assert rel(out["K"], ref["K"]) < TOL64
    assert abs(out["Ex"][0] - ref["Ex"]) < TOL64 * abs(ref["Ex"])


@pytest.mark.parametrize("n", [24, 30, 32, 36, 40, 48])
@pytest.mark.parametrize("mode", ["symmetric", "fftfreq"])
def test_every_specialised_grid_size_fp64(n, mode):
    """Each compile-time grid specialisation against the oracle (small k-mesh and basis)."""
    prob = W.small_problem(kmesh=(1, 2, 1), grid=(n, n, n), nocc=3, counts=(2, 1, 1), seed=40 + n)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, mode)
    plan, out = run_gpu(prob, C, mode)
    ph = periodic_phase(prob)
    assert rel(plan.intermediate("W").cpu().numpy(), ref["W"] * ph[:, None, :]) < TOL64
    assert rel(out["Kmi"], ref["Kmi"]) < TOL64
    assert abs(out["Ex"][0] - ref["Ex"]) < TOL64 * abs(ref["Ex"])


@pytest.mark.parametrize("n", [24, 32, 36, 40, 48])
@pytest.mark.parametrize("precision", [pkg.PREC_FP32, pkg.PREC_FP32_SPLIT])
@pytest.mark.parametrize("mode", ["symmetric", "fftfreq"])
def test_register_and_lds_transforms_agree(n, precision, mode):
    """The register-resident line FFTs (complex64 plans) against the LDS Stockham passes
    on the same inputs.  Both compute the same sums in a different order, so they agree
    to complex64 rounding: 2e-6 relative (a few ulps accumulated over log N butterfly
    levels and 8 orbitals)."""
    prob = W.small_problem(kmesh=(1, 2, 2), grid=(n, n, n), nocc=8, counts=(2, 2, 1), seed=60 + n)
    C = W.random_coefficients(prob)
    tol = 2e-6
    p_lds, o_lds = run_gpu(prob, C, mode, precision=precision, flags=pkg.FLAG_LDS_FFT)
    w_lds = p_lds.intermediate("W").cpu().numpy()
    for flags in (0, pkg.FLAG_REG_FFT_ALL):
        p_reg, o_reg = run_gpu(prob, C, mode, precision=precision, flags=flags)
        w_reg = p_reg.intermediate("W").cpu().numpy()
        assert rel(w_reg, w_lds) < tol, flags
        assert rel(o_reg["Kmi"], o_lds["Kmi"]) < tol, flags
        assert abs(o_reg["Ex"][0] - o_lds["Ex"][0]) < tol * abs(o_lds["Ex"][0]), flags


@pytest.mark.parametrize("n", [24, 32, 36, 40, 48])
@pytest.mark.parametrize("mode", ["symmetric", "fftfreq"])
def test_register_path_fp32_split_against_oracle(n, mode):
    """Complex64 plans on cubic grids, with the LDS passes and with the register-resident
    passes: checked against the FP64 oracle to the reduced-precision bars
    (|dE_x| <= 1e-6 Eh, max |dK~| <= 1e-5)."""
    prob = W.small_problem(kmesh=(1, 2, 2), grid=(n, n, n), nocc=8, counts=(2, 2, 1), seed=80 + n)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, mode)
    for flags in (0, pkg.FLAG_REG_FFT_ALL):
        _, out = run_gpu(prob, C, mode, precision=pkg.PREC_FP32_SPLIT, flags=flags)
        assert abs(out["Ex"][0] - ref["Ex"]) <= 1e-6, flags
        assert np.max(np.abs(out["K"] - ref["K"])) <= 1e-5, flags


@pytest.mark.parametrize("kernel,omega", [(W.KERNEL_COULOMB, 0.0), (W.KERNEL_ERF_LR, 0.3)])
@pytest.mark.parametrize("mode", ["symmetric", "fftfreq"])
def test_madelung_mode_against_oracle(kernel, omega, mode):
    """OCCRIK_FLAG_MADELUNG: G + q = 0 term from the supercell's Ewald Madelung constant
    (computed on the host by the library, by the oracle in its own code)."""
    prob = W.small_problem(kmesh=(2, 1, 3), grid=(12, 10, 9), nocc=3, kernel=kernel, omega=omega)
    C = W.random_coefficients(prob)
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
    ref = occrik.build(prob, C, chi=chi, nyquist=mode, madelung=True,
                       domega=kernel == W.KERNEL_ERF_LR)
    plan, out = run_gpu(prob, C, mode, flags=pkg.FLAG_MADELUNG)
    assert rel(out["Kmi"], ref["Kmi"]) < TOL64
    assert rel(out["K"], ref["K"]) < TOL64
    assert abs(out["Ex"][0] - ref["Ex"]) < TOL64 * abs(ref["Ex"])
    if kernel == W.KERNEL_ERF_LR and mode == "symmetric":
        _, dw = plan.grad(1.0, want_C=False, want_omega=True)
        assert abs(dw - ref["dEx_domega"]) < TOL64 * abs(ref["dEx_domega"])


def test_madelung_mode_s_gaussian_closed_form_on_gpu():
    """-sqrt(a/pi) - pi/(2 a L^3): the image term xi / 2L removed by the Madelung G = 0 value."""
    L, alpha = 18.0, 0.6
    cell = W.cubic_cell(L, [(0.5, 0.5, 0.5)])
    basis = W.Basis(np.zeros(1, np.int32), np.zeros(1, np.int32), np.array([alpha]))
    prob = W.Problem("sgauss", cell, basis, (1, 1, 1), (60, 60, 60), 1, seed=0)
    C = np.ones((1, 1, 1), dtype=complex)
    exact = -np.sqrt(alpha / np.pi) - np.pi / (2 * alpha * L ** 3)
    for precision, tol in ((pkg.PREC_FP64, 1e-10), (pkg.PREC_FP32_SPLIT, 1e-6)):
        _, out = run_gpu(prob, C, "symmetric", precision=precision, flags=pkg.FLAG_MADELUNG)
        assert abs(out["Ex"][0] - exact) < tol, precision


@pytest.mark.parametrize("n", [24, 30, 32, 36, 40, 48])
@pytest.mark.parametrize("precision", [pkg.PREC_FP32, pkg.PREC_FP32_SPLIT])
@pytest.mark.parametrize("mode", ["symmetric", "fftfreq"])
def test_every_specialised_grid_size_complex64(n, precision, mode):
    """The complex64 pair passes of each compiled grid size (LDS two-stage kernels)
    against the FP64 oracle to the reduced-precision bars: |dE_x| <= 1e-6 Eh,
    max |dK~| <= 1e-5, and K_{mu j} within 1e-5 relative."""
    prob = W.small_problem(kmesh=(1, 2, 1), grid=(n, n, n), nocc=3, counts=(2, 1, 1), seed=40 + n)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, mode)
    _, out = run_gpu(prob, C, mode, precision=precision, flags=pkg.FLAG_LDS_FFT)
    assert abs(out["Ex"][0] - ref["Ex"]) <= 1e-6
    assert np.max(np.abs(out["K"] - ref["K"])) <= 1e-5
    assert rel(out["Kmi"], ref["Kmi"]) < 1e-5


@pytest.mark.parametrize("n,precision", [(24, pkg.PREC_FP64), (30, pkg.PREC_FP64), (48, pkg.PREC_FP64),
                                         (30, pkg.PREC_FP32), (36, pkg.PREC_FP32_SPLIT)])
def test_omega_gradient_on_specialised_grids(n, precision):
    """d E_x / d omega from the forward-only sweep (pass 2 without the inverse
    transforms) on compiled grid sizes, against the oracle's Parseval form."""
    prob = W.small_problem(kmesh=(1, 2, 1), grid=(n, n, n), nocc=3, counts=(2, 1, 1), seed=90 + n,
                           kernel=W.KERNEL_ERF_LR, omega=0.35)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, "symmetric")
    plan, _ = run_gpu(prob, C, "symmetric", precision=precision)
    _, dw = plan.grad(1.0, want_C=False, want_omega=True)
    tol = TOL64 if precision == pkg.PREC_FP64 else 1e-5
    assert abs(dw - ref["dEx_domega"]) < tol * abs(ref["dEx_domega"])


@pytest.mark.parametrize("case", [
    dict(kmesh=(1, 1, 1), grid=(1, 8, 6), nocc=1, counts=(2, 1)),        # Gamma only, one orbital, extent 1
    dict(kmesh=(1, 1, 2), grid=(2, 3, 4), nocc=2, counts=(1, 1)),        # the smallest grid extents
    dict(kmesh=(1, 2, 1), grid=(10, 9, 8), nocc=16, counts=(2, 2, 1)),   # the largest orbital count
    dict(kmesh=(1, 1, 2), grid=(12, 10, 9), nocc=8, counts=(1, 1)),      # N_ao = nocc (square C)
    dict(kmesh=(1, 1, 1), grid=(48, 48, 48), nocc=8, counts=(1, 1)),     # one k-point on a compiled size
])
@pytest.mark.parametrize("mode", ["symmetric", "fftfreq"])
def test_degenerate_shapes(case, mode):
    """Edge shapes the method admits: a single k-point and orbital, grid extents of 1
    and 2, 16 occupied orbitals, as many orbitals as AOs."""
    case = dict(case)
    prob = W.small_problem(seed=5 + case["nocc"], **case)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, mode)
    _, out = run_gpu(prob, C, mode)
    assert rel(out["Kmi"], ref["Kmi"]) < TOL64
    assert rel(out["K"], ref["K"]) < TOL64
    assert abs(out["Ex"][0] - ref["Ex"]) < TOL64 * abs(ref["Ex"])
    _, o32 = run_gpu(prob, C, mode, precision=pkg.PREC_FP32_SPLIT)
    assert abs(o32["Ex"][0] - ref["Ex"]) <= 1e-6
    assert np.max(np.abs(o32["K"] - ref["K"])) <= 1e-5


@pytest.mark.parametrize("nocc,n,kmesh", [(1, 24, (1, 2, 2)), (2, 36, (2, 1, 1)), (7, 32, (1, 1, 2)),
                                          (6, 40, (1, 2, 1)), (9, 36, (1, 1, 2)), (12, 30, (2, 1, 1)),
                                          (16, 24, (1, 2, 1))])
@pytest.mark.parametrize("precision", [pkg.PREC_FP64, pkg.PREC_FP32_SPLIT])
def test_compiled_sizes_with_other_orbital_counts(nocc, n, kmesh, precision):
    """Rows of the diagonal block with 1..nocc stored pairs, odd and even orbital
    counts and partial orbital groups in the compiled-size pair passes; 9 to 16
    occupied orbitals (the largest count a plan takes) run pass 3 with 16 orbital
    lines per column."""
    prob = W.small_problem(kmesh=kmesh, grid=(n, n, n), nocc=nocc, counts=(2, 2, 1), seed=120 + nocc)
    C = W.random_coefficients(prob)
    ref = oracle_result(prob, C, "symmetric")
    _, out = run_gpu(prob, C, "symmetric", precision=precision)
    if precision == pkg.PREC_FP64:
        assert rel(out["Kmi"], ref["Kmi"]) < TOL64
        assert abs(out["Ex"][0] - ref["Ex"]) < TOL64 * abs(ref["Ex"])
    else:
        assert abs(out["Ex"][0] - ref["Ex"]) <= 1e-6
        assert np.max(np.abs(out["K"] - ref["K"])) <= 1e-5
