"""GPU tests of the reduced-precision modes, the adjoint, error paths, invariants
and the ragged batch entry point, all through the C ABI."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import collocation, occrik
import paper_2207_09028_amd as pkg
from paper_2207_09028_amd import OccrikError
from paper_2207_09028_amd.autograd import exchange_energy
from paper_2207_09028_amd.plan import BatchGraph, Plan, PlanSpec, build_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu_required():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


_cache = {}


def ref_for(prob, C, nyquist="symmetric", domega=False):
    key = (prob.name, prob.grid, prob.kmesh, prob.nocc, prob.kernel, prob.omega, nyquist, prob.seed, domega)
    if key not in _cache:
        chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
        _cache[key] = occrik.build(prob, C, chi=chi, nyquist=nyquist, domega=domega)
    return _cache[key]


# ----------------------------------------------------------------------------
# reduced precision
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("prec", [pkg.PREC_FP32, pkg.PREC_FP32_SPLIT])
@pytest.mark.parametrize("name", ["tiny", "small"])
def test_reduced_precision_meets_the_accuracy_gate(prec, name):
    """|dE_x| <= 1e-6 E_h and max|dK~| <= 1e-5 against the FP64 oracle."""
    prob = W.make_problem(name) if name != "small" else W.small_problem()
    C = W.random_coefficients(prob)
    ref = ref_for(prob, C)
    plan = Plan(PlanSpec.from_problem(prob, precision=prec))
    out = plan.build(torch.from_numpy(C).to("cuda"))
    dE = abs(float(out["Ex"][0]) - ref["Ex"])
    dK = float(np.max(np.abs(out["K"].cpu().numpy() - ref["K"])))
    print(name, prec, "dEx", dE, "max dK", dK)
    assert dE <= 1e-6
    assert dK <= 1e-5


# ----------------------------------------------------------------------------
# adjoint
# ----------------------------------------------------------------------------

def test_gradient_in_C_is_2K_over_Nk_and_matches_finite_differences():
    prob = W.small_problem()
    C = W.random_coefficients(prob)
    ref = ref_for(prob, C)
    plan = Plan(PlanSpec.from_problem(prob))
    Ct = torch.from_numpy(C).to("cuda")
    plan.build(Ct)
    g, _ = plan.grad(1.0, want_C=True)
    g = g.cpu().numpy()
    assert rel(g, occrik.energy_gradient_C(ref["Kmi"], prob.nk)) < 1e-10
    rng = np.random.default_rng(7)
    h = 1e-5
    for _ in range(4):
        k, mu, i = int(rng.integers(prob.nk)), int(rng.integers(prob.nao)), int(rng.integers(prob.nocc))
        for unit, part in ((1.0, "re"), (1j, "im")):
            Cp = C.copy(); Cp[k, mu, i] += h * unit
            Cm = C.copy(); Cm[k, mu, i] -= h * unit
            ep = float(plan.build(torch.from_numpy(Cp).to("cuda"), want_K=False)["Ex"][0])
            em = float(plan.build(torch.from_numpy(Cm).to("cuda"), want_K=False)["Ex"][0])
            fd = (ep - em) / (2 * h)
            an = g[k, mu, i].real if part == "re" else g[k, mu, i].imag
            assert abs(fd - an) < 1e-7 * max(1.0, abs(an)) + 1e-9


@pytest.mark.parametrize("kind", [W.KERNEL_ERF_LR, W.KERNEL_TRUNC_ERF_LR])
def test_gradient_in_omega_matches_oracle_and_finite_differences(kind):
    prob = W.small_problem(kernel=kind, omega=0.3)
    C = W.random_coefficients(prob)
    ref = ref_for(prob, C, domega=True)
    plan = Plan(PlanSpec.from_problem(prob))
    Ct = torch.from_numpy(C).to("cuda")
    plan.build(Ct, want_K=False)
    _, dw = plan.grad(1.0, want_C=False, want_omega=True)
    assert abs(dw - ref["dEx_domega"]) < 1e-10 * abs(ref["dEx_domega"])
    h = 1e-4
    plan.set_omega(0.3 + h)
    ep = float(plan.build(Ct, want_K=False)["Ex"][0])
    plan.set_omega(0.3 - h)
    em = float(plan.build(Ct, want_K=False)["Ex"][0])
    assert abs((ep - em) / (2 * h) - dw) < 1e-7 * abs(dw)


def test_autograd_function_backward():
    prob = W.small_problem(kernel=W.KERNEL_ERF_LR, omega=0.35)
    C = W.random_coefficients(prob)
    plan = Plan(PlanSpec.from_problem(prob))
    Ct = torch.from_numpy(C).to("cuda").requires_grad_(True)
    w = torch.tensor(0.35, dtype=torch.float64, requires_grad=True)
    E = exchange_energy(plan, Ct, w)
    (3.0 * E).backward()
    ref = ref_for(prob, C, domega=True)
    assert abs(float(E) - ref["Ex"]) < 1e-10 * abs(ref["Ex"])
    assert rel(Ct.grad.cpu().numpy(), 3.0 * occrik.energy_gradient_C(ref["Kmi"], prob.nk)) < 1e-10
    assert abs(float(w.grad) - 3.0 * ref["dEx_domega"]) < 1e-10 * abs(3.0 * ref["dEx_domega"])


def test_autograd_backward_after_another_forward_on_the_same_plan_raises():
    """The adjoint reads the plan's last build: a second forward on the same plan before
    the first backward would hand C1 the gradient of C2, so backward refuses; one plan
    per live graph gives both gradients."""
    prob = W.small_problem(kernel=W.KERNEL_ERF_LR, omega=0.35)
    prob2 = W.small_problem(kernel=W.KERNEL_ERF_LR, omega=0.35, seed=6)   # same cell, other coefficients
    C1 = W.random_coefficients(prob)
    C2 = W.random_coefficients(prob2)
    plan = Plan(PlanSpec.from_problem(prob))
    t1 = torch.from_numpy(C1).to("cuda").requires_grad_(True)
    t2 = torch.from_numpy(C2).to("cuda").requires_grad_(True)
    E = exchange_energy(plan, t1) + exchange_energy(plan, t2)
    with pytest.raises(RuntimeError, match="built again"):
        E.backward()
    other = Plan(PlanSpec.from_problem(prob))
    t1.grad = None
    t2.grad = None
    E = exchange_energy(plan, t1) + exchange_energy(other, t2)
    E.backward()
    assert rel(t1.grad.cpu().numpy(), occrik.energy_gradient_C(ref_for(prob, C1)["Kmi"], prob.nk)) < 1e-10
    assert rel(t2.grad.cpu().numpy(), occrik.energy_gradient_C(ref_for(prob2, C2)["Kmi"], prob.nk)) < 1e-10


def test_grad_before_build_is_a_state_error():
    prob = W.small_problem()
    plan = Plan(PlanSpec.from_problem(prob))
    with pytest.raises(OccrikError) as e:
        plan.grad(1.0)
    assert e.value.status == 7


# ----------------------------------------------------------------------------
# invariants
# ----------------------------------------------------------------------------

def test_invariants_on_gpu_outputs():
    prob = W.make_problem("tiny")
    C = W.random_coefficients(prob)
    plan = Plan(PlanSpec.from_problem(prob))
    out = plan.build(torch.from_numpy(C).to("cuda"))
    K = out["K"].cpu().numpy()
    Kmi = out["Kmi"].cpu().numpy()
    assert np.max(np.abs(K - K.conj().transpose(0, 2, 1))) < 1e-13 * np.max(np.abs(K))
    assert rel(np.einsum("kab,kbi->kai", K, C), Kmi) < 1e-11
    # gauge invariance: C -> C U_k leaves K~ and E_x unchanged
    rng = np.random.default_rng(5)
    U = np.stack([np.linalg.qr(rng.standard_normal((prob.nocc, prob.nocc)) +
                               1j * rng.standard_normal((prob.nocc, prob.nocc)))[0] for _ in range(prob.nk)])
    C2 = np.einsum("kmi,kij->kmj", C, U)
    out2 = plan.build(torch.from_numpy(C2).to("cuda"))
    assert rel(out2["K"].cpu().numpy(), K) < 1e-11
    assert abs(float(out2["Ex"][0]) - float(out["Ex"][0])) < 1e-12 * abs(float(out["Ex"][0]))


# ----------------------------------------------------------------------------
# error paths (forced from the host; every kernel still exits normally)
# ----------------------------------------------------------------------------

def test_singular_occupied_block_reports_not_pd_with_k():
    prob = W.small_problem()
    C = W.random_coefficients(prob)
    C[3, :, 1] = 0.0                             # empty orbital at k = 3: K_ij(3) has a zero row and column
    plan = Plan(PlanSpec.from_problem(prob))
    with pytest.raises(OccrikError) as e:
        plan.build(torch.from_numpy(C).to("cuda"))
    assert e.value.status == 4 and e.value.k == 3
    # the plan stays usable
    C2 = W.random_coefficients(prob)
    plan.build(torch.from_numpy(C2).to("cuda"))


def test_nonfinite_coefficients_are_reported():
    prob = W.small_problem()
    C = W.random_coefficients(prob)
    C[1, 2, 0] = np.nan
    plan = Plan(PlanSpec.from_problem(prob))
    with pytest.raises(OccrikError) as e:
        plan.build(torch.from_numpy(C).to("cuda"))
    assert e.value.status == 5
    with pytest.raises(OccrikError) as e:
        plan.build_host(C)
    assert e.value.status == 5


def test_memory_budget_too_small_reports_oom():
    prob = W.small_problem()
    with pytest.raises(OccrikError) as e:
        Plan(PlanSpec.from_problem(prob, mem_budget=1 << 16))
    assert e.value.status == 3


# ----------------------------------------------------------------------------
# ragged batch
# ----------------------------------------------------------------------------

def _ragged_batch(precisions=(pkg.PREC_FP32,)):
    probs = [W.small_problem(kmesh=(2, 1, 1), grid=(12, 10, 9), nocc=3, seed=1),
             W.small_problem(kmesh=(1, 2, 2), grid=(8, 9, 10), nocc=2, counts=(1, 1, 1), seed=2),
             W.small_problem(kmesh=(2, 2, 1), grid=(24, 24, 24), nocc=4, counts=(2, 2, 1), seed=3),
             W.small_problem(kmesh=(1, 1, 3), grid=(16, 15, 12), nocc=5, counts=(2, 2, 1), seed=4),
             W.small_problem(kmesh=(2, 2, 2), grid=(20, 20, 20), nocc=3, seed=5)]
    out = []
    for i, p in enumerate(probs):
        prec = precisions[i % len(precisions)]
        out.append((p, W.random_coefficients(p), prec))
    return out


def test_batch_graph_replays_match_eager_builds():
    """A ragged batch recorded as one HIP graph: every replay, with other device work and
    synchronisations in between, reproduces the single eager builds bitwise."""
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        items = _ragged_batch((pkg.PREC_FP32, pkg.PREC_FP64, pkg.PREC_FP32_SPLIT))
        plans, Cs, Ks, Kmis, Es, ref = [], [], [], [], [], []
        for p, C, prec in items:
            plan = Plan(PlanSpec.from_problem(p, precision=prec))
            Ct = torch.from_numpy(C).to("cuda")
            r = plan.build(Ct)
            ref.append({k: v.clone() for k, v in r.items()})
            plans.append(plan)
            Cs.append(Ct)
            Ks.append(torch.empty_like(r["K"]))
            Kmis.append(torch.empty_like(r["Kmi"]))
            Es.append(torch.empty(1, dtype=torch.float64, device="cuda"))
        graph = BatchGraph(plans, Cs, Ks=Ks, Kmis=Kmis, Exs=Es)
        for rep in range(3):
            for t in Ks + Kmis + Es:
                t.fill_(float("nan"))
            x = torch.randn(1 << 20, device="cuda")
            (x * x).sum().item()                       # unrelated eager work between replays
            graph.launch()
            side.synchronize()
            for i, (K, Kmi, E) in enumerate(zip(Ks, Kmis, Es)):
                assert torch.equal(K, ref[i]["K"]), (rep, i)
                assert torch.equal(Kmi, ref[i]["Kmi"]), (rep, i)
                assert torch.equal(E, ref[i]["Ex"]), (rep, i)
            for plan in plans:
                plan.status()
        graph.close()


def test_fused_batch_rounds_match_single_builds():
    """With occrik_batch_create_fused, plans that share a kernel form run their pair
    passes in fused rounds, one launch per pass for several cells: complex64 plans on 24^3 (FP32 and FP32-split, one with
    conduction-band columns) with the 8-line pass 3, complex64 plans with 10 occupied
    orbitals on 24^3 (16-line pass 3) and FP64 plans on 30^3, on ragged k-meshes; one
    plan on a run-time grid builds whole beside them.  Every replay equals the single
    eager builds bitwise, and the FP64 members match the oracle."""
    cases = [
        (dict(kmesh=(2, 1, 2), grid=(24, 24, 24), nocc=3, seed=61), dict(precision=pkg.PREC_FP32_SPLIT)),
        (dict(kmesh=(1, 2, 1), grid=(24, 24, 24), nocc=4, counts=(2, 2, 1), seed=62), dict(precision=pkg.PREC_FP32)),
        (dict(kmesh=(2, 2, 1), grid=(24, 24, 24), nocc=5, counts=(2, 2, 1), seed=63),
         dict(precision=pkg.PREC_FP32_SPLIT, nocc=3, nvir=2)),
        (dict(kmesh=(1, 1, 2), grid=(24, 24, 24), nocc=10, counts=(2, 2, 1), seed=64),
         dict(precision=pkg.PREC_FP32_SPLIT)),
        (dict(kmesh=(2, 1, 1), grid=(24, 24, 24), nocc=10, counts=(2, 2, 1), seed=65), dict(precision=pkg.PREC_FP32)),
        (dict(kmesh=(1, 2, 2), grid=(30, 30, 30), nocc=3, seed=66), dict(precision=pkg.PREC_FP64)),
        (dict(kmesh=(2, 1, 1), grid=(30, 30, 30), nocc=4, counts=(2, 1, 1), seed=67), dict(precision=pkg.PREC_FP64)),
        (dict(kmesh=(2, 1, 1), grid=(12, 10, 9), nocc=3, seed=68), dict(precision=pkg.PREC_FP32_SPLIT)),
    ]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        probs, plans, Cs, Ks, Kmis, Es, ref = [], [], [], [], [], [], []
        for pk, sk in cases:
            prob = W.small_problem(**pk)
            C = torch.from_numpy(W.random_coefficients(prob)).to("cuda")
            plan = Plan(PlanSpec.from_problem(prob, **sk))
            r = plan.build(C)
            ref.append({k: v.clone() for k, v in r.items()})
            probs.append(prob)
            plans.append(plan)
            Cs.append(C)
            Ks.append(torch.empty_like(r["K"]))
            Kmis.append(torch.empty_like(r["Kmi"]))
            Es.append(torch.empty(1, dtype=torch.float64, device="cuda"))
        graph = BatchGraph(plans, Cs, Ks=Ks, Kmis=Kmis, Exs=Es, fused=True)
        assert graph.fused == 7
        plain = BatchGraph(plans, Cs, Ks=Ks, Kmis=Kmis, Exs=Es)
        assert plain.fused == 0
        plain.close()
        for rep in range(2):
            for t in Ks + Kmis + Es:
                t.fill_(float("nan"))
            graph.launch()
            side.synchronize()
            for i in range(len(cases)):
                plans[i].status()
                assert torch.equal(Ks[i], ref[i]["K"]), (rep, i)
                assert torch.equal(Kmis[i], ref[i]["Kmi"]), (rep, i)
                assert torch.equal(Es[i], ref[i]["Ex"]), (rep, i)
        graph.close()
    for i in (5, 6):
        prob = probs[i]
        chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
        o = occrik.build(prob, Cs[i].cpu().numpy(), chi=chi, nyquist="symmetric")
        K = ref[i]["K"].cpu().numpy()
        assert np.max(np.abs(K - o["K"])) < 1e-10 * np.max(np.abs(o["K"])), i
        assert abs(float(ref[i]["Ex"][0]) - o["Ex"]) < 1e-10 * abs(o["Ex"]), i


def test_grouped_pass1_rows_match_single_row_launches():
    """Pass 1 holds four summed orbitals per workgroup on launches of at least 4096
    single-row workgroups and one below that; fused batch rounds always take one row.
    Two FP64 plans on 24^3 with a 4x4x4 mesh (5 occupied + 1 band: row groups of 4 and
    1; 6 occupied: groups of 4 and 2) run their first rows grouped in single builds;
    the fused batch of the same plans must give the same K~, K_{mu j} and E_x to
    rounding."""
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        specs = [(dict(kmesh=(4, 4, 4), grid=(24, 24, 24), nocc=6, counts=(2, 1, 1), seed=151), dict(nocc=5, nvir=1)),
                 (dict(kmesh=(4, 4, 4), grid=(24, 24, 24), nocc=6, counts=(2, 1, 1), seed=152), dict())]
        plans, Cs, Ks, Kmis, Es, ref = [], [], [], [], [], []
        for pk, sk in specs:
            prob = W.small_problem(**pk)
            C = torch.from_numpy(W.random_coefficients(prob)).to("cuda")
            plan = Plan(PlanSpec.from_problem(prob, precision=pkg.PREC_FP64, **sk))
            r = plan.build(C)
            ref.append({k: v.clone() for k, v in r.items()})
            plans.append(plan)
            Cs.append(C)
            Ks.append(torch.empty_like(r["K"]))
            Kmis.append(torch.empty_like(r["Kmi"]))
            Es.append(torch.empty(1, dtype=torch.float64, device="cuda"))
        graph = BatchGraph(plans, Cs, Ks=Ks, Kmis=Kmis, Exs=Es, fused=True)
        assert graph.fused == 2
        graph.launch()
        side.synchronize()
        for i in range(len(specs)):
            plans[i].status()
            for got, want in ((Ks[i], ref[i]["K"]), (Kmis[i], ref[i]["Kmi"])):
                g, w = got.cpu().numpy(), want.cpu().numpy()
                assert np.max(np.abs(g - w)) <= 1e-12 * np.max(np.abs(w)), i
            e, w = float(Es[i][0]), float(ref[i]["Ex"][0])
            assert abs(e - w) <= 1e-12 * abs(w), i
        graph.close()


def test_grouped_pass1_prefetch_wave_complex64():
    """In complex64 the four-row pass-1 launches carry an extra wave that loads a later
    workgroup's held orbitals into L2 and passes the same barriers as the other waves.
    FP32 plans on 24^3 and 30^3 (the latter's planes are not a whole number of 128-byte
    lines; fused rounds group plans of one grid, so two of each) with a 4x4x4 mesh run
    their first rows grouped in single builds (groups of 4 and 1, 4 and 2, 4 and 3) and
    single rows in the fused batch; both must agree with each other and with the FP64
    build at the reduced-precision bars (|dE_x| <= 1e-6 Eh, max |dK~| <= 1e-5)."""
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        specs = [(dict(kmesh=(4, 4, 4), grid=(24, 24, 24), nocc=6, counts=(2, 1, 1), seed=153), dict(nocc=5, nvir=1)),
                 (dict(kmesh=(4, 4, 4), grid=(24, 24, 24), nocc=6, counts=(2, 1, 1), seed=155), dict()),
                 (dict(kmesh=(4, 4, 4), grid=(30, 30, 30), nocc=7, counts=(2, 1, 1), seed=154), dict()),
                 (dict(kmesh=(4, 4, 4), grid=(30, 30, 30), nocc=6, counts=(2, 1, 1), seed=156), dict())]
        plans, Cs, Ks, Kmis, Es, ref, ref64 = [], [], [], [], [], [], []
        for pk, sk in specs:
            prob = W.small_problem(**pk)
            C = torch.from_numpy(W.random_coefficients(prob)).to("cuda")
            r64 = Plan(PlanSpec.from_problem(prob, precision=pkg.PREC_FP64, **sk)).build(C)
            ref64.append({k: v.cpu().numpy() for k, v in r64.items()})
            plan = Plan(PlanSpec.from_problem(prob, precision=pkg.PREC_FP32, **sk))
            r = plan.build(C)
            ref.append({k: v.cpu().numpy() for k, v in r.items()})
            plans.append(plan)
            Cs.append(C)
            Ks.append(torch.empty_like(r["K"]))
            Kmis.append(torch.empty_like(r["Kmi"]))
            Es.append(torch.empty(1, dtype=torch.float64, device="cuda"))
        graph = BatchGraph(plans, Cs, Ks=Ks, Kmis=Kmis, Exs=Es, fused=True)
        assert graph.fused == 4
        graph.launch()
        side.synchronize()
        for i in range(len(specs)):
            plans[i].status()
            K, Kmi, e = Ks[i].cpu().numpy(), Kmis[i].cpu().numpy(), float(Es[i][0])
            for got in (ref[i], {"K": K, "Kmi": Kmi, "Ex": np.array([e])}):
                assert abs(float(got["Ex"][0]) - float(ref64[i]["Ex"][0])) <= 1e-6, i
                assert np.max(np.abs(got["K"] - ref64[i]["K"])) <= 1e-5, i
                assert np.max(np.abs(got["Kmi"] - ref64[i]["Kmi"])) <= 1e-5, i
            # grouped and single-row complex64 passes differ only in rounding order
            assert np.max(np.abs(K - ref[i]["K"])) <= 1e-6 * np.max(np.abs(ref[i]["K"])), i
        graph.close()


def test_ragged_batch_equals_single_builds_bitwise():
    probs = [W.small_problem(kmesh=(2, 1, 1), grid=(12, 10, 9), nocc=3, seed=1),
             W.small_problem(kmesh=(1, 2, 2), grid=(8, 9, 10), nocc=2, counts=(1, 1, 1), seed=2),
             W.small_problem(kmesh=(2, 2, 1), grid=(24, 24, 24), nocc=4, counts=(2, 2, 1), seed=3)]
    plans, Cs, Ks, Es, singles = [], [], [], [], []
    for p in probs:
        C = W.random_coefficients(p)
        plan = Plan(PlanSpec.from_problem(p, precision=pkg.PREC_FP32))
        Ct = torch.from_numpy(C).to("cuda")
        singles.append(plan.build(Ct))
        plans.append(plan)
        Cs.append(Ct)
        Ks.append(torch.empty_like(singles[-1]["K"]))
        Es.append(torch.empty(1, dtype=torch.float64, device="cuda"))
    build_batch(plans, Cs, Ks=Ks, Exs=Es)
    torch.cuda.synchronize()
    for s, K, E in zip(singles, Ks, Es):
        assert torch.equal(s["K"], K) and torch.equal(s["Ex"], E)


# ----------------------------------------------------------------------------
# integral-direct plans (Sec. II.E, Alg. 4): chi~ collocated per build
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("precision", [pkg.PREC_FP64, pkg.PREC_FP32, pkg.PREC_FP32_SPLIT])
def test_integral_direct_is_bitwise_the_stored_build(precision):
    """Forced direct mode and the stored mode run the same per-point collocation and the
    same partial-sum chunks of the contraction, so every output is bitwise equal."""
    prob = W.make_problem("tiny")
    C = torch.from_numpy(W.random_coefficients(prob)).to("cuda")
    stored = Plan(PlanSpec.from_problem(prob, precision=precision))
    direct = Plan(PlanSpec.from_problem(prob, precision=precision, flags=pkg.FLAG_DIRECT))
    assert stored.query().integral_direct == 0 and direct.query().integral_direct == 1
    assert direct.query().bytes_chi == 0
    a = stored.build(C)
    b = direct.build(C)
    for key in ("K", "Kmi", "Ex"):
        assert torch.equal(a[key], b[key]), key
    with pytest.raises(pkg.OccrikError):
        direct.intermediate("chi")


@pytest.mark.parametrize("precision", [pkg.PREC_FP64, pkg.PREC_FP32_SPLIT])
def test_integral_direct_with_more_chunks_than_filled_is_bitwise_the_stored_build(precision):
    """64 contraction chunks asked for on 12 x 10 x 9 points: chunks of 32 points fill
    only 34 of them, and the plan keeps those 34 (an empty trailing chunk would never be
    written by the direct contraction, which launches the chunks a collocation chunk
    covers).  Direct and stored builds stay bitwise equal, and both match the oracle."""
    prob = W.small_problem(kmesh=(2, 1, 2), grid=(12, 10, 9), nocc=3, seed=41)
    Cn = W.random_coefficients(prob)
    C = torch.from_numpy(Cn).to("cuda")
    stored = Plan(PlanSpec.from_problem(prob, precision=precision, contract_chunks=64))
    direct = Plan(PlanSpec.from_problem(prob, precision=precision, contract_chunks=64, flags=pkg.FLAG_DIRECT))
    assert stored.query().contract_chunks == 34 and direct.query().contract_chunks == 34
    for _ in range(2):
        a = stored.build(C)
        b = direct.build(C)
        for key in ("K", "Kmi", "Ex"):
            assert torch.equal(a[key], b[key]), key
    ref = occrik.build(prob, Cn, nyquist="symmetric")
    tol = 1e-10 * abs(ref["Ex"]) if precision == pkg.PREC_FP64 else 1e-6
    assert abs(float(b["Ex"][0]) - ref["Ex"]) < tol


def test_integral_direct_switches_on_by_memory_budget_with_several_chunks():
    """A budget too small for the stored chi~ turns the direct mode on by itself, with
    chunks of a budget-eighth (three collocation chunks here); the FP64 result is still
    bitwise the stored one and matches the oracle."""
    prob = W.make_problem("tiny")
    Cn = W.random_coefficients(prob)
    C = torch.from_numpy(Cn).to("cuda")
    stored = Plan(PlanSpec.from_problem(prob, kbatch=2))
    budget = 64 << 20
    assert stored.query().bytes_chi + stored.query().bytes_workspace > budget
    direct = Plan(PlanSpec.from_problem(prob, kbatch=2, mem_budget=budget))
    info = direct.query()
    assert info.integral_direct == 1
    assert info.colloc_chunk < info.ng
    assert info.bytes_chi + info.bytes_workspace <= budget
    a = stored.build(C)
    b = direct.build(C)
    for key in ("K", "Kmi", "Ex"):
        assert torch.equal(a[key], b[key]), key
    ref = occrik.build(prob, Cn, nyquist="symmetric")
    assert abs(float(b["Ex"][0]) - ref["Ex"]) < 1e-10 * abs(ref["Ex"])


# ----------------------------------------------------------------------------
# conduction-band extension (Sec. II.D): nvir extra columns treated exactly
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("grid,nocc,nvir,mode", [((12, 10, 9), 2, 2, "symmetric"), ((12, 10, 9), 2, 2, "fftfreq"),
                                                 ((24, 24, 24), 3, 3, "symmetric"),
                                                 ((24, 24, 24), 5, 6, "symmetric")])
def test_conduction_bands_match_oracle(grid, nocc, nvir, mode):
    prob = W.small_problem(kmesh=(2, 1, 2), grid=grid, nocc=nocc + nvir, counts=(2, 2, 1), seed=17)
    C = W.random_coefficients(prob)
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
    ref = occrik.build(prob, C, chi=chi, nyquist=mode, nvir=nvir)
    spec = PlanSpec.from_problem(prob, nocc=nocc, nvir=nvir, nyquist=1 if mode == "symmetric" else 0)
    plan = Plan(spec)
    out = plan.build(torch.from_numpy(C).to("cuda"))
    Kmi, K, Ex = out["Kmi"].cpu().numpy(), out["K"].cpu().numpy(), float(out["Ex"][0])
    assert np.max(np.abs(Kmi - ref["Kmi"])) < 1e-10 * np.max(np.abs(ref["Kmi"]))
    assert np.max(np.abs(K - ref["K"])) < 1e-10 * np.max(np.abs(ref["K"]))
    assert abs(Ex - ref["Ex"]) < 1e-10 * abs(ref["Ex"])
    # gradient: (2/N_k) K_{mu j} on the occupied columns, zero on the bands
    g, _ = plan.grad(1.0)
    g = g.cpu().numpy()
    assert np.max(np.abs(g[:, :, :nocc] - 2.0 / prob.nk * ref["Kmi"][:, :, :nocc])) < 1e-10 * np.max(np.abs(g))
    assert np.all(g[:, :, nocc:] == 0)
    # FP32-split on the same plan inputs
    p32 = Plan(PlanSpec.from_problem(prob, nocc=nocc, nvir=nvir, precision=pkg.PREC_FP32_SPLIT,
                                     nyquist=1 if mode == "symmetric" else 0))
    o32 = p32.build(torch.from_numpy(C).to("cuda"))
    assert abs(float(o32["Ex"][0]) - ref["Ex"]) <= 1e-6
    assert np.max(np.abs(o32["K"].cpu().numpy() - ref["K"])) <= 1e-5


def test_conduction_bands_leave_energy_and_omega_derivative_unchanged():
    prob = W.small_problem(kmesh=(2, 1, 1), grid=(12, 10, 9), nocc=5, kernel=W.KERNEL_ERF_LR, omega=0.3)
    C = W.random_coefficients(prob)
    Ct = torch.from_numpy(C).to("cuda")
    occ = Plan(PlanSpec.from_problem(prob, nocc=3))
    ext = Plan(PlanSpec.from_problem(prob, nocc=3, nvir=2))
    e_occ = float(occ.build(Ct[:, :, :3].contiguous())["Ex"][0])
    e_ext = float(ext.build(Ct)["Ex"][0])
    assert abs(e_occ - e_ext) < 1e-12 * abs(e_occ)
    _, d_occ = occ.grad(1.0, want_C=False, want_omega=True)
    _, d_ext = ext.grad(1.0, want_C=False, want_omega=True)
    assert abs(d_occ - d_ext) < 1e-11 * abs(d_occ)


# ----------------------------------------------------------------------------
# autotuner: k batch, pair-transform form and contraction chunks chosen by timing
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("precision,grid", [(pkg.PREC_FP64, (24, 24, 24)), (pkg.PREC_FP32, (24, 24, 24)),
                                            (pkg.PREC_FP32_SPLIT, (12, 10, 9))])
def test_autotuned_plan_builds_bitwise_as_the_explicit_settings(precision, grid):
    prob = W.small_problem(kmesh=(2, 2, 2), grid=grid, nocc=4, counts=(2, 1, 1), seed=31)
    C = W.random_coefficients(prob)
    Ct = torch.from_numpy(C).to("cuda")
    plan = Plan(PlanSpec.from_problem(prob, precision=precision))
    before = plan.query()
    res = plan.autotune(Ct)
    info = plan.query()
    assert info.tuned == 1 and res["builds"] >= 2
    assert info.kbatch == res["kbatch"] and info.contract_chunks == res["contract_chunks"]
    assert 1 <= res["kbatch"] <= before.kbatch and 1 <= res["contract_chunks"] <= 64
    assert res["ms_best"] <= res["ms_initial"]
    if res["reg_fft"]:
        assert precision != pkg.PREC_FP64
    out = plan.build(Ct)
    flags = pkg.FLAG_REG_FFT_ALL if res["reg_fft"] else pkg.FLAG_LDS_FFT
    ref = Plan(PlanSpec.from_problem(prob, precision=precision, kbatch=res["kbatch"], flags=flags,
                                     contract_chunks=res["contract_chunks"])).build(Ct)
    for key in ("K", "Kmi", "Ex"):
        assert torch.equal(out[key], ref[key]), key
    if precision == pkg.PREC_FP64:
        chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
        oref = occrik.build(prob, C, chi=chi, nyquist="symmetric")
        assert abs(float(out["Ex"][0]) - oref["Ex"]) < 1e-10 * abs(oref["Ex"])


def test_autotune_keeps_the_settings_the_parameters_fix():
    prob = W.small_problem(kmesh=(2, 1, 2), grid=(24, 24, 24), nocc=3, counts=(2, 1, 1), seed=32)
    Ct = torch.from_numpy(W.random_coefficients(prob)).to("cuda")
    plan = Plan(PlanSpec.from_problem(prob, precision=pkg.PREC_FP32, kbatch=1, flags=pkg.FLAG_LDS_FFT,
                                      contract_chunks=3))
    res = plan.autotune(Ct)
    assert (res["kbatch"], res["reg_fft"], res["contract_chunks"]) == (1, 0, 3)
    direct = Plan(PlanSpec.from_problem(prob, precision=pkg.PREC_FP32, flags=pkg.FLAG_DIRECT))
    n0 = direct.query().contract_chunks
    res = direct.autotune(Ct)
    assert res["contract_chunks"] == n0
    # a tuned integral-direct plan still equals its stored counterpart bitwise
    stored = Plan(PlanSpec.from_problem(prob, precision=pkg.PREC_FP32, kbatch=res["kbatch"],
                                        flags=pkg.FLAG_REG_FFT_ALL if res["reg_fft"] else pkg.FLAG_LDS_FFT))
    a, b = direct.build(Ct), stored.build(Ct)
    assert torch.equal(a["Kmi"], b["Kmi"]) and torch.equal(a["Ex"], b["Ex"])
