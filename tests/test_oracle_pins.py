"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test ties one oracle function to the paper or to mathematics: a brute-force
evaluation of the defining sums, an analytic closed form, an identity the paper
states, a second algorithm the paper gives, or finite differences.  The
``test_mutation_*`` tests plant plausible mistakes in the oracle (on the CPU)
and check that a pin catches each of them.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import collocation, conventional, kernels, occrik
from oracle import lattice as olat


# ----------------------------------------------------------------------------
# P1: the discrete plane-wave fit and potential (eqs. aodf, Vrao, VGao)
# ----------------------------------------------------------------------------

def test_pair_potential_matches_brute_force_sums():
    """Z^G and V(r) evaluated as explicit sums over grid points and G vectors."""
    rng = np.random.default_rng(0)
    cell = W.Cell(np.array([[5.0, 0.3, 0.0], [0.2, 4.0, 0.4], [0.0, -0.5, 6.0]]), np.zeros((1, 3)))
    grid = (5, 6, 4)
    kmesh = (2, 3, 1)
    geo = occrik.Geometry(cell, kmesh, grid)
    rho = rng.standard_normal(geo.ng) + 1j * rng.standard_normal(geo.ng)
    k2, k1 = 4, 1                      # q = k2 - k1 nonzero, fractional, unwrapped
    V, _ = occrik.pair_potentials(geo, rho[None, :], k2, k1, kernels.COULOMB, 0.0)
    q = geo.kcart[k2] - geo.kcart[k1]
    omega = abs(np.linalg.det(cell.lattice))
    dv = omega / geo.ng
    Vb = np.zeros(geo.ng, dtype=complex)
    # the DFT's G set: integer triples in numpy frequency order
    ms = [olat.fft_indices(n) for n in grid]
    for m1 in ms[0]:
        for m2 in ms[1]:
            for m3 in ms[2]:
                G = m1 * geo.recip[0] + m2 * geo.recip[1] + m3 * geo.recip[2]
                Gq = G + q
                Z = np.sum(rho * np.exp(-1j * (geo.r @ Gq))) * dv / omega
                x2 = float(Gq @ Gq)
                f = 0.0 if x2 == 0.0 else 4 * np.pi / x2
                Vb += f * Z * np.exp(1j * (geo.r @ Gq))
    assert np.max(np.abs(V[0] - Vb)) < 1e-12 * np.max(np.abs(Vb))


def test_nyquist_convention_is_numpy_fftfreq():
    assert list(olat.fft_indices(6)) == [0, 1, 2, -3, -2, -1]
    assert list(olat.fft_indices(5)) == [0, 1, 2, -2, -1]


# ----------------------------------------------------------------------------
# P2: collocation (Sec. II.A Bloch sum) and normalisation
# ----------------------------------------------------------------------------

def _phi_scalar(x, y, z, alpha, a, b, c):
    l = a + b + c
    df = lambda n: 1 if n <= 1 else n * df(n - 2)
    nrm = (2 * alpha / math.pi) ** 0.75 * (4 * alpha) ** (l / 2) / math.sqrt(df(2 * a - 1) * df(2 * b - 1) * df(2 * c - 1))
    return nrm * x ** a * y ** b * z ** c * math.exp(-alpha * (x * x + y * y + z * z))


def test_collocation_matches_scalar_bloch_sum():
    prob = W.small_problem(kmesh=(2, 2, 1), grid=(6, 5, 4), counts=(1, 1, 1), amin=0.4, amax=2.0)
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, 1e-12)
    lat = prob.cell.lattice
    kc = olat.kpoints_cartesian(lat, prob.kmesh)
    r = olat.grid_points(lat, prob.grid)
    centers = prob.cell.atoms_frac @ lat
    labels = collocation.ao_labels(prob.basis)
    rng = np.random.default_rng(1)
    n_img = 9
    for _ in range(12):
        k = int(rng.integers(prob.nk))
        mu = int(rng.integers(prob.nao))
        n = int(rng.integers(prob.ng))
        s, ic = labels[mu]
        l = int(prob.basis.shell_l[s])
        a, b, c = collocation.cartesian_powers(l)[ic]
        alpha = float(prob.basis.shell_exp[s])
        R = centers[prob.basis.shell_atom[s]]
        tot = 0j
        for t1 in range(-n_img, n_img + 1):
            for t2 in range(-n_img, n_img + 1):
                for t3 in range(-n_img, n_img + 1):
                    T = t1 * lat[0] + t2 * lat[1] + t3 * lat[2]
                    x = r[n] - R - T
                    tot += np.exp(1j * kc[k] @ T) * _phi_scalar(x[0], x[1], x[2], alpha, a, b, c)
        assert abs(chi[k, mu, n] - tot) < 1e-11


# eq. occmo in the streamed form that writes the paper-sized stored values: chi is
# formed for a slab of grid points at a time and contracted with C at once.  Pinned
# against the composition of the two pinned functions above (collocation, then
# occmo) on whole, ragged and one-point slabs, and against scalar Bloch sums
# contracted with C by hand at sampled points (independent of ``collocate``).

def _streamed_reference():
    prob = W.small_problem(kmesh=(2, 2, 1), grid=(6, 5, 4), nocc=2, counts=(1, 1, 1), amin=0.4, amax=2.0)
    C = W.random_coefficients(prob)
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, 1e-12)
    return prob, C, occrik.occupied_orbitals(chi, C)


def _scalar_orbital(prob, C, k, i, n, n_img=9):
    lat = prob.cell.lattice
    kc = olat.kpoints_cartesian(lat, prob.kmesh)[k]
    r = olat.grid_points(lat, prob.grid)[n]
    centers = prob.cell.atoms_frac @ lat
    tot = 0j
    for mu, (s, ic) in enumerate(collocation.ao_labels(prob.basis)):
        a, b, c = collocation.cartesian_powers(int(prob.basis.shell_l[s]))[ic]
        alpha = float(prob.basis.shell_exp[s])
        R = centers[prob.basis.shell_atom[s]]
        chi = 0j
        for t1 in range(-n_img, n_img + 1):
            for t2 in range(-n_img, n_img + 1):
                for t3 in range(-n_img, n_img + 1):
                    T = t1 * lat[0] + t2 * lat[1] + t3 * lat[2]
                    x = r - R - T
                    chi += np.exp(1j * kc @ T) * _phi_scalar(x[0], x[1], x[2], alpha, a, b, c)
        tot += C[k, mu, i] * chi
    return tot


def _check_streamed(prob, C, ref, chunk):
    psi = collocation.occupied_orbitals_streamed(prob.cell, prob.basis, prob.kmesh, prob.grid, C, 1e-12,
                                                 chunk=chunk)
    assert psi.shape == ref.shape
    assert np.max(np.abs(psi - ref)) <= 1e-13 * np.max(np.abs(ref))
    return psi


@pytest.mark.parametrize("chunk", [7, 1, 1000])
def test_streamed_orbitals_equal_collocation_then_occmo(chunk):
    """chunk 7: slabs smaller than the 120-point grid with a one-point last slab;
    chunk 1: one point per slab; chunk 1000: the whole grid in one slab."""
    prob, C, ref = _streamed_reference()
    _check_streamed(prob, C, ref, chunk)


def test_streamed_orbitals_match_scalar_bloch_sums():
    prob, C, _ = _streamed_reference()
    psi = collocation.occupied_orbitals_streamed(prob.cell, prob.basis, prob.kmesh, prob.grid, C, 1e-12, chunk=7)
    rng = np.random.default_rng(3)
    for _ in range(4):
        k, i, n = int(rng.integers(prob.nk)), int(rng.integers(prob.nocc)), int(rng.integers(prob.ng))
        assert abs(psi[k, i, n] - _scalar_orbital(prob, C, k, i, n)) < 1e-11


def test_mutation_streamed_orbitals_without_bloch_phase_fail(monkeypatch):
    prob, C, ref = _streamed_reference()        # reference from the unmutated path
    orig = olat.kpoints_fractional
    monkeypatch.setattr(collocation.lat_mod, "kpoints_fractional", lambda km: 0.0 * orig(km))
    with pytest.raises(AssertionError):
        _check_streamed(prob, C, ref, 7)


def test_mutation_streamed_orbitals_with_transposed_coefficients_fail():
    prob, C, ref = _streamed_reference()
    Ct = C.copy()
    Ct[:, :2, :] = C[:, :2, :][:, ::-1, :]       # two AO rows exchanged: a wrong mu index
    with pytest.raises(AssertionError):
        _check_streamed(prob, Ct, ref, 7)


def test_isolated_gto_is_normalised():
    """int |phi|^2 = 1 for s, p, d, f components, by quadrature in a large cell."""
    cell = W.cubic_cell(14.0, [(0.5, 0.5, 0.5)])
    basis = W.Basis(np.zeros(4, np.int32), np.array([0, 1, 2, 3], np.int32), np.array([1.1, 0.9, 0.8, 0.7]))
    grid = (48, 48, 48)
    chi = collocation.collocate(cell, basis, (1, 1, 1), grid, 1e-14)
    dv = 14.0 ** 3 / np.prod(grid)
    norms = dv * np.sum(np.abs(chi[0]) ** 2, axis=1)
    assert np.max(np.abs(norms - 1.0)) < 1e-9


def test_grid_overlap_matches_analytic_overlap():
    """dV chi^H chi on a fine grid equals the analytic lattice-summed overlap S_k
    (Obara-Saika, computed by the input generator, not by the oracle)."""
    prob = W.small_problem(kmesh=(2, 1, 2), grid=(36, 36, 36), counts=(2, 1, 1), amin=0.25, amax=1.2)
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, 1e-13)
    dv = abs(np.linalg.det(prob.cell.lattice)) / prob.ng
    Sg = dv * np.einsum("kmn,kln->kml", chi.conj(), chi)
    Sa = W.overlap_k(prob)
    assert np.max(np.abs(Sg - Sa)) < 1e-9


def test_shell_extent_solves_threshold():
    for alpha, l in [(0.05, 0), (0.5, 1), (3.0, 2), (50.0, 3)]:
        r = collocation.shell_extent(alpha, l, 1e-12)
        nmax = (2 * alpha / math.pi) ** 0.75 * (4 * alpha) ** (l / 2)
        assert abs(nmax * r ** l * math.exp(-alpha * r * r) / 1e-12 - 1.0) < 1e-9


# ----------------------------------------------------------------------------
# P3: normalisation of K and E_x: a single s-Gaussian in a large cubic cell
# ----------------------------------------------------------------------------

def _madelung_sc(L):
    """Simple-cubic Madelung constant xi (E = -xi / 2L for unit charges) by Ewald summation."""
    eta = 2.0 / L
    real = 0.0
    rec = 0.0
    n = 6
    for i in range(-n, n + 1):
        for j in range(-n, n + 1):
            for k in range(-n, n + 1):
                if i == j == k == 0:
                    continue
                d = L * math.sqrt(i * i + j * j + k * k)
                real += math.erfc(eta * d) / d
                g2 = (2 * math.pi / L) ** 2 * (i * i + j * j + k * k)
                rec += math.exp(-g2 / (4 * eta * eta)) / g2
    vol = L ** 3
    e = 0.5 * (real + 4 * math.pi / vol * rec - 2 * eta / math.sqrt(math.pi) - math.pi / (eta * eta * vol))
    return -2.0 * L * e


def test_madelung_constant_value():
    assert abs(_madelung_sc(1.0) - 2.837297479) < 1e-8


def test_s_gaussian_exchange_closed_form():
    """E_x = -sqrt(a/pi) + xi/(2L) - pi/(2 a L^3) for one normalised s function (G=0 term zeroed)."""
    L, alpha = 18.0, 0.6
    cell = W.cubic_cell(L, [(0.5, 0.5, 0.5)])
    basis = W.Basis(np.zeros(1, np.int32), np.zeros(1, np.int32), np.array([alpha]))
    prob = W.Problem("sgauss", cell, basis, (1, 1, 1), (60, 60, 60), 1, seed=0)
    C = np.ones((1, 1, 1), dtype=complex)
    res = occrik.build(prob, C, want_k=False)
    xi = _madelung_sc(1.0)
    exact = -math.sqrt(alpha / math.pi) + xi / (2 * L) - math.pi / (2 * alpha * L ** 3)
    assert abs(res["Ex"] - exact) < 1e-10


# ----------------------------------------------------------------------------
# P4/P5: occ-RI-K reproduces the conventional exchange on occupied quantities
# ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small():
    prob = W.small_problem()
    C = W.random_coefficients(prob)
    res = occrik.build(prob, C, parseval=True)
    return prob, C, res


def test_occrik_equals_mo_k_on_occupied_quantities(small):
    prob, C, res = small
    Kc = conventional.mo_k(prob, C, res["chi"])
    KC = np.einsum("kab,kbi->kai", Kc, C)
    assert np.max(np.abs(KC - res["Kmi"])) < 1e-12
    CKC = np.einsum("kai,kab,kbj->kij", C.conj(), Kc, C)
    assert np.max(np.abs(CKC - res["Kij"])) < 1e-12
    e_conv = np.real(np.einsum("kii->", CKC)) / (2 * prob.nk)
    assert abs(e_conv - res["Ex"]) < 1e-13


def test_ao_k_equals_mo_k(small):
    prob, C, res = small
    Km = conventional.mo_k(prob, C, res["chi"])
    Ka = conventional.ao_k(prob, C, res["chi"])
    assert np.max(np.abs(Ka - Km)) < 1e-12
    # conventional K is Hermitian and negative semidefinite
    assert np.max(np.abs(Km - Km.conj().transpose(0, 2, 1))) < 1e-13
    for k in range(prob.nk):
        assert np.max(np.linalg.eigvalsh(0.5 * (Km[k] + Km[k].conj().T))) < 1e-12


def test_trace_energy_equals_parseval_energy(small):
    _, _, res = small
    assert abs(res["Ex"] - res["Ex_parseval"]) < 1e-13 * abs(res["Ex"])


# ----------------------------------------------------------------------------
# P6: assembly
# ----------------------------------------------------------------------------

def test_assembly_identities(small):
    prob, C, res = small
    K = res["K"]
    assert np.max(np.abs(np.einsum("kab,kbi->kai", K, C) - res["Kmi"])) < 1e-12
    assert np.max(np.abs(np.einsum("kai,kab,kbj->kij", C.conj(), K, C) - res["Kij"])) < 1e-12
    assert np.max(np.abs(K - K.conj().transpose(0, 2, 1))) < 1e-14
    for k in range(prob.nk):
        assert np.max(np.linalg.eigvalsh(-0.5 * (res["Kij"][k] + res["Kij"][k].conj().T))) > 0


def test_gauge_invariance(small):
    prob, C, res = small
    rng = np.random.default_rng(3)
    U = np.empty((prob.nk, prob.nocc, prob.nocc), dtype=complex)
    for k in range(prob.nk):
        q, _ = np.linalg.qr(rng.standard_normal((prob.nocc, prob.nocc)) + 1j * rng.standard_normal((prob.nocc, prob.nocc)))
        U[k] = q
    C2 = np.einsum("kmi,kij->kmj", C, U)
    res2 = occrik.build(prob, C2, chi=res["chi"])
    assert np.max(np.abs(res2["K"] - res["K"])) < 1e-12
    assert abs(res2["Ex"] - res["Ex"]) < 1e-13
    assert np.max(np.abs(res2["Kij"] - np.einsum("kai,kab,kbj->kij", U.conj(), res["Kij"], U))) < 1e-12


def test_projector_form_agrees_on_occupied_space(small):
    prob, C, res = small
    chi = res["chi"]
    dv = abs(np.linalg.det(prob.cell.lattice)) / prob.ng
    S = dv * np.einsum("kmn,kln->kml", chi.conj(), chi)
    # orthonormalise C in the grid metric so that C^H S C = 1 holds exactly
    Cg = np.empty_like(C)
    for k in range(prob.nk):
        M = C[k].conj().T @ S[k] @ C[k]
        w, U = np.linalg.eigh(M)
        Cg[k] = C[k] @ (U / np.sqrt(w)) @ U.conj().T
    r = occrik.build(prob, Cg, chi=chi)
    KP = occrik.assemble_projector(r["Kmi"], r["Kij"], S, Cg)
    assert np.max(np.abs(np.einsum("kab,kbi->kai", KP, Cg) - r["Kmi"])) < 1e-12


def test_projector_form_is_the_full_exchange_in_a_complete_basis():
    """With as many orbitals as AOs and C^H S C = 1 (grid metric), SC = C^-H, so the
    three terms of eq. occrikop are K, K and K and the projector form is the
    conventional AO-RI-K matrix (Alg. 1, eq. aok) itself, computed without K_mu."""
    prob = W.small_problem(kmesh=(2, 1, 1), grid=(8, 7, 6), nocc=10, counts=(2, 1), amin=0.4, amax=2.0)
    assert prob.nocc == prob.nao
    C = W.random_coefficients(prob)
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
    dv = abs(np.linalg.det(prob.cell.lattice)) / prob.ng
    S = dv * np.einsum("kmn,kln->kml", chi.conj(), chi)
    Cg = np.empty_like(C)
    for k in range(prob.nk):
        M = C[k].conj().T @ S[k] @ C[k]
        w, U = np.linalg.eigh(M)
        Cg[k] = C[k] @ (U / np.sqrt(w)) @ U.conj().T
    r = occrik.build(prob, Cg, chi=chi, want_k=False)
    KP = occrik.assemble_projector(r["Kmi"], r["Kij"], S, Cg)
    Ka = conventional.ao_k(prob, Cg, chi)
    assert np.max(np.abs(Ka)) > 0.1
    assert np.max(np.abs(KP - Ka)) < 1e-12


# ----------------------------------------------------------------------------
# P7: gradients
# ----------------------------------------------------------------------------

def test_energy_is_the_same_in_both_nyquist_modes(small):
    """The Nyquist modes differ only by the antisymmetric part of the discrete
    exchange form, which vanishes on the diagonal: E_x is identical, K is not."""
    prob, C, res = small
    rs = occrik.build(prob, C, chi=res["chi"], nyquist="symmetric")
    assert abs(rs["Ex"] - res["Ex"]) < 1e-14 * abs(res["Ex"])
    assert np.max(np.abs(rs["Kmi"] - res["Kmi"])) > 1e-8


def test_energy_gradient_in_C_by_finite_differences(small):
    """dE_x/dRe C + i dE_x/dIm C = (2/N_k) K C holds exactly for the symmetric-Nyquist K
    (the symmetric part of the discrete exchange form); the fftfreq-mode K misses it
    by a Nyquist-plane term."""
    prob, C, res = small
    rs = occrik.build(prob, C, chi=res["chi"], nyquist="symmetric", want_k=False)
    g = occrik.energy_gradient_C(rs["Kmi"], prob.nk)
    g_fftfreq = occrik.energy_gradient_C(res["Kmi"], prob.nk)
    worst_fftfreq = 0.0
    rng = np.random.default_rng(4)
    h = 1e-5
    for _ in range(6):
        k = int(rng.integers(prob.nk)); mu = int(rng.integers(prob.nao)); i = int(rng.integers(prob.nocc))
        for part, unit in (("re", 1.0), ("im", 1j)):
            Cp = C.copy(); Cp[k, mu, i] += h * unit
            Cm = C.copy(); Cm[k, mu, i] -= h * unit
            ep = occrik.build(prob, Cp, chi=res["chi"], want_k=False)["Ex"]
            em = occrik.build(prob, Cm, chi=res["chi"], want_k=False)["Ex"]
            fd = (ep - em) / (2 * h)
            an = g[k, mu, i].real if part == "re" else g[k, mu, i].imag
            assert abs(fd - an) < 1e-8 * max(1.0, abs(an)) + 1e-9
            af = g_fftfreq[k, mu, i].real if part == "re" else g_fftfreq[k, mu, i].imag
            worst_fftfreq = max(worst_fftfreq, abs(fd - af))
    assert worst_fftfreq > 1e-8


@pytest.mark.parametrize("kind,madelung", [(W.KERNEL_ERF_LR, False), (W.KERNEL_TRUNC_ERF_LR, False),
                                           (W.KERNEL_ERF_LR, True)])
def test_energy_derivative_in_omega_by_finite_differences(kind, madelung):
    prob = W.small_problem(kernel=kind, omega=0.3)
    C = W.random_coefficients(prob)
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, 1e-12)
    res = occrik.build(prob, C, chi=chi, want_k=False, domega=True, madelung=madelung)
    h = 2e-5          # the Madelung mode's pi / w^2 term has a large third derivative
    ep = occrik.build(prob, C, chi=chi, want_k=False, omega=0.3 + h, madelung=madelung)["Ex"]
    em = occrik.build(prob, C, chi=chi, want_k=False, omega=0.3 - h, madelung=madelung)["Ex"]
    fd = (ep - em) / (2 * h)
    assert abs(fd - res["dEx_domega"]) < 1e-7 * abs(fd)


# ----------------------------------------------------------------------------
# P8: kernels
# ----------------------------------------------------------------------------

def test_kernel_limits_and_additivity():
    w = 0.37
    x2 = np.array([0.0, 1e-9, 0.3, 2.0, 17.0])
    sr = kernels.kernel_values(x2, kernels.ERFC_SR, w)
    lr = kernels.kernel_values(x2, kernels.ERF_LR, w)
    co = kernels.kernel_values(x2, kernels.COULOMB, w)
    assert abs(sr[0] - math.pi / w ** 2) < 1e-14
    assert abs(sr[1] - math.pi / w ** 2) < 1e-8 * math.pi / w ** 2      # continuity at x -> 0
    assert np.max(np.abs((sr + lr - co)[2:] / co[2:])) < 1e-14
    assert co[0] == 0.0 and lr[0] == 0.0
    # omega derivatives against central differences of the kernels themselves
    for kind in (kernels.ERF_LR, kernels.ERFC_SR):
        d = kernels.kernel_domega(x2[2:], kind, w)
        fd = (kernels.kernel_values(x2[2:], kind, w + 1e-6) - kernels.kernel_values(x2[2:], kind, w - 1e-6)) / 2e-6
        assert np.max(np.abs(d - fd)) < 1e-6 * np.max(np.abs(d))


def test_exchange_is_additive_in_the_kernel(small):
    """E[erfc] + E[erf] = E[1/r] + the energy of the G+q=0 term pi/w^2 of the short-range kernel."""
    prob, C, res = small
    w = 0.45
    e_sr = occrik.build(prob, C, chi=res["chi"], want_k=False, kind=kernels.ERFC_SR, omega=w)["Ex"]
    e_lr = occrik.build(prob, C, chi=res["chi"], want_k=False, kind=kernels.ERF_LR, omega=w)["Ex"]
    e_c = res["Ex"]
    geo = occrik.Geometry(prob.cell, prob.kmesh, prob.grid)
    psi = res["psi"]
    g0 = 0.0
    for k in range(prob.nk):                       # q = 0 blocks only
        for i in range(prob.nocc):
            for j in range(prob.nocc):
                u0 = np.sum(np.conj(psi[k, i]) * psi[k, j])
                g0 += (math.pi / w ** 2) * abs(u0) ** 2
    e0 = -geo.omega_cell / (2 * prob.nk ** 2 * prob.ng ** 2) * g0
    assert abs(e_sr + e_lr - e_c - e0) < 1e-12


# ----------------------------------------------------------------------------
# P9: k-mesh calculation equals the Gamma-point supercell calculation
# ----------------------------------------------------------------------------

def _supercell(prob, C):
    M = prob.kmesh
    lat = prob.cell.lattice
    sc_lat = lat * np.array(M)[:, None]
    cells = [(a, b, c) for a in range(M[0]) for b in range(M[1]) for c in range(M[2])]
    atoms, sa, sl, se = [], [], [], []
    for L in cells:
        for ia, f in enumerate(prob.cell.atoms_frac):
            atoms.append((np.array(L) + f) / np.array(M))
            idx = len(atoms) - 1
            for s in range(prob.basis.nshell):
                if prob.basis.shell_atom[s] == ia:
                    sa.append(idx); sl.append(prob.basis.shell_l[s]); se.append(prob.basis.shell_exp[s])
    basis = W.Basis(np.array(sa, np.int32), np.array(sl, np.int32), np.array(se))
    # AO order of the supercell: cell L, then the unit cell's AO order
    nao = prob.nao
    kf = olat.kpoints_fractional(M)
    Csc = np.zeros((1, nao * len(cells), prob.nk * prob.nocc), dtype=complex)
    for ic, L in enumerate(cells):
        ph = np.exp(2j * np.pi * (kf @ np.array(L)))
        for k in range(prob.nk):
            Csc[0, ic * nao:(ic + 1) * nao, k * prob.nocc:(k + 1) * prob.nocc] = C[k] * ph[k] / math.sqrt(prob.nk)
    grid = tuple(int(g * m) for g, m in zip(prob.grid, M))
    sc = W.Problem("sc", W.Cell(sc_lat, np.array(atoms)), basis, (1, 1, 1), grid, prob.nk * prob.nocc, seed=0)
    return sc, Csc


def test_kmesh_equals_gamma_supercell():
    prob = W.small_problem(kmesh=(2, 1, 2), grid=(16, 16, 16), nocc=2, counts=(2, 1), amin=0.35, amax=0.9)
    C = W.random_coefficients(prob)
    e_k = occrik.build(prob, C, want_k=False)["Ex"]
    sc, Csc = _supercell(prob, C)
    e_sc = occrik.build(sc, Csc, want_k=False)["Ex"]
    assert abs(e_sc / prob.nk - e_k) < 1e-9 * abs(e_k)


# ----------------------------------------------------------------------------
# Nyquist modes: the conjugate-pair identity the symmetric mode makes exact
# ----------------------------------------------------------------------------

def test_symmetric_nyquist_makes_conjugate_pairs_exact():
    prob = W.small_problem(kmesh=(2, 2, 1), grid=(8, 6, 4))
    C = W.random_coefficients(prob)
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, 1e-12)
    psi = occrik.occupied_orbitals(chi, C)
    geo = occrik.Geometry(prob.cell, prob.kmesh, prob.grid)
    k1, k2, i, j = 1, 2, 0, 2
    for mode, expect_exact in (("symmetric", True), ("fftfreq", False)):
        Va, _ = occrik.pair_potentials(geo, (np.conj(psi[k1, i]) * psi[k2, j])[None], k2, k1, 0, 0.0, mode)
        Vb, _ = occrik.pair_potentials(geo, (np.conj(psi[k2, j]) * psi[k1, i])[None], k1, k2, 0, 0.0, mode)
        d = np.max(np.abs(Va - np.conj(Vb)))
        if expect_exact:
            assert d < 1e-13 * np.max(np.abs(Va))
        else:
            assert d > 1e-8 * np.max(np.abs(Va))


# ----------------------------------------------------------------------------
# mutation tests: a plausible mistake anywhere in the oracle fails a pin
# ----------------------------------------------------------------------------

def test_mutation_dropped_volume_element_fails_madelung(monkeypatch):
    orig = occrik.contract
    monkeypatch.setattr(occrik, "contract", lambda geo, chi, Wt: orig(geo, chi, Wt) / geo.dv)
    with pytest.raises(AssertionError):
        test_s_gaussian_exchange_closed_form()


def test_mutation_wrong_momentum_sign_fails_supercell(monkeypatch):
    orig = occrik.Geometry.kernel_on_grid

    def flipped(self, k2, k1, kind, omega, nyquist="fftfreq", derivative=False):
        return orig(self, k1, k2, kind, omega, nyquist, derivative)

    monkeypatch.setattr(occrik.Geometry, "kernel_on_grid", flipped)
    with pytest.raises(AssertionError):
        test_kmesh_equals_gamma_supercell()


def test_mutation_transposed_coefficients_fail_mo_identity(monkeypatch, small):
    monkeypatch.setattr(occrik, "occupied_block", lambda C, Kmi: np.einsum("kmi,kmj->kij", C, Kmi))
    prob, C, res = small
    r = occrik.build(prob, C, chi=res["chi"], want_k=False)
    Kc = conventional.mo_k(prob, C, res["chi"])
    CKC = np.einsum("kai,kab,kbj->kij", C.conj(), Kc, C)
    assert np.max(np.abs(CKC - r["Kij"])) > 1e-6


def test_mutation_missing_bloch_phase_fails_overlap(monkeypatch):
    orig = olat.kpoints_fractional
    monkeypatch.setattr(collocation.lat_mod, "kpoints_fractional", lambda km: 0.0 * orig(km))
    with pytest.raises(AssertionError):
        test_grid_overlap_matches_analytic_overlap()


# ----------------------------------------------------------------------------
# Truncated Coulomb kernel (Sec. II.A, Spencer-Alavi): 1/r cut off at R_c with
# 4 pi R_c^3 / 3 = N_k Omega
# ----------------------------------------------------------------------------

def test_truncated_coulomb_kernel_matches_radial_quadrature():
    """f(G) = int_{r < R_c} e^{-iG.r} / r d^3r = (4 pi / G) int_0^{R_c} sin(G r) dr, by quadrature."""
    from scipy.integrate import quad
    rc = 7.3
    g = np.array([1e-7, 0.05, 0.4, 1.7, 6.1, 23.0])
    f = kernels.kernel_values(g * g, kernels.TRUNC_COULOMB, 0.0, rc)
    for gi, fi in zip(g, f):
        val, _ = quad(lambda r: 4.0 * math.pi * math.sin(gi * r) / gi, 0.0, rc, limit=400)
        assert abs(fi - val) < 1e-10 * max(abs(val), 1.0), (gi, fi, val)
    f0 = kernels.kernel_values(np.array([0.0]), kernels.TRUNC_COULOMB, 0.0, rc)[0]
    assert abs(f0 - 2.0 * math.pi * rc * rc) < 1e-12 * f0          # int_{r<R_c} d^3r / r
    assert kernels.truncation_radius(8, 10.0) ** 3 * 4.0 * math.pi / 3.0 == pytest.approx(80.0, rel=1e-14)


def _isolated_gaussian_exchange_truncated(L, n, kmesh, alpha=0.6):
    cell = W.cubic_cell(L, [(0.5, 0.5, 0.5)])
    basis = W.Basis(np.zeros(1, np.int32), np.zeros(1, np.int32), np.array([alpha]))
    prob = W.Problem("sgauss", cell, basis, kmesh, (n, n, n), 1, seed=0, kernel=kernels.TRUNC_COULOMB)
    C = W.random_coefficients(prob)
    return occrik.build(prob, C, want_k=False)["Ex"]


def test_truncated_coulomb_gives_the_isolated_gaussian_exchange_at_gamma():
    """With the cut-off sphere inside one cell's reach no periodic image interacts, so one
    normalised s-Gaussian has E_x = -sqrt(a/pi) exactly (no Madelung term), G = 0 included."""
    alpha = 0.6
    assert abs(_isolated_gaussian_exchange_truncated(24.0, 64, (1, 1, 1), alpha) + math.sqrt(alpha / math.pi)) < 1e-12


def test_truncated_coulomb_gives_the_isolated_gaussian_exchange_on_a_kmesh():
    """A lattice of well separated s-Gaussians (spacing 8 bohr, 3x3x3 k-points): R_c now comes
    from the 24 bohr k-mesh supercell, and the per-cell E_x is again -sqrt(a/pi)."""
    alpha = 0.6
    assert abs(_isolated_gaussian_exchange_truncated(8.0, 28, (3, 3, 3), alpha) + math.sqrt(alpha / math.pi)) < 1e-12


def test_mutation_truncation_radius_without_kpoints_fails(monkeypatch):
    """R_c from Omega alone (N_k dropped) cuts each Gaussian's own tail: the k-mesh pin's
    1e-12 bar catches it by orders of magnitude."""
    real = kernels.truncation_radius
    monkeypatch.setattr(kernels, "truncation_radius", lambda nk, vol: real(1, vol))
    alpha = 0.6
    err = abs(_isolated_gaussian_exchange_truncated(8.0, 28, (3, 3, 3), alpha) + math.sqrt(alpha / math.pi))
    assert err > 1e-9


# ----------------------------------------------------------------------------
# Truncated long-range kernel (eq. lrtrunc): erf(w r)/r cut off at R_c
# ----------------------------------------------------------------------------

def test_truncated_long_range_kernel_matches_radial_quadrature():
    """f(G) = (4 pi / G) int_0^{R_c} erf(w r) sin(G r) dr and f(0) = 4 pi int_0^{R_c} r erf(w r) dr,
    by quadrature of the real-space definition (independent of the complex error function)."""
    from scipy.integrate import quad
    for w, rc in ((0.3, 15.8), (1.1, 3.0), (0.05, 8.0)):
        g = np.array([0.0, 0.3, 0.7, 2.0, 5.3])
        f = kernels.kernel_values(g * g, kernels.TRUNC_ERF_LR, w, rc)
        for gi, fi in zip(g, f):
            if gi == 0.0:
                val, _ = quad(lambda r: 4.0 * math.pi * r * math.erf(w * r), 0.0, rc, limit=400)
            else:
                val, _ = quad(lambda r: 4.0 * math.pi * math.erf(w * r) * math.sin(gi * r) / gi, 0.0, rc,
                              limit=2000)
            assert abs(fi - val) < 1e-11 * max(abs(val), 1.0), (w, rc, gi, fi, val)


def test_truncated_long_range_limits():
    """For w R_c >> 1 the cut-off erf(w r)/r is the cut-off 1/r minus erfc(w r)/r (whose tail
    beyond R_c is negligible), so f_trunc_LR = f_trunc_Coulomb - f_SR; d f/dw matches central
    differences."""
    rc = 9.0
    x2 = np.array([0.0, 0.04, 1.3, 7.0, 40.0])
    for w in (6.0, 60.0):
        lr = kernels.kernel_values(x2, kernels.TRUNC_ERF_LR, w, rc)
        co = kernels.kernel_values(x2, kernels.TRUNC_COULOMB, 0.0, rc)
        sr = kernels.kernel_values(x2, kernels.ERFC_SR, w)
        assert np.max(np.abs(lr - (co - sr))) < 1e-11 * np.max(np.abs(co)), w
    w = 0.37
    d = kernels.kernel_domega(x2, kernels.TRUNC_ERF_LR, w, rc)
    fd = (kernels.kernel_values(x2, kernels.TRUNC_ERF_LR, w + 1e-5, rc)
          - kernels.kernel_values(x2, kernels.TRUNC_ERF_LR, w - 1e-5, rc)) / 2e-5
    assert np.max(np.abs(d - fd)) < 1e-6 * np.max(np.abs(d))


def _isolated_gaussian_exchange(L, n, kmesh, kind, omega, alpha=0.6):
    cell = W.cubic_cell(L, [(0.5, 0.5, 0.5)])
    basis = W.Basis(np.zeros(1, np.int32), np.zeros(1, np.int32), np.array([alpha]))
    prob = W.Problem("sgauss", cell, basis, kmesh, (n, n, n), 1, seed=0, kernel=kind, omega=omega)
    C = W.random_coefficients(prob)
    return occrik.build(prob, C, want_k=False)["Ex"]


@pytest.mark.parametrize("L,n,kmesh", [(24.0, 64, (1, 1, 1)), (8.0, 28, (3, 3, 3))])
def test_truncated_long_range_gives_the_isolated_attenuated_exchange(L, n, kmesh):
    """One normalised s-Gaussian, no image inside the sphere: E_x is the attenuated self-exchange
    -sqrt(mu/pi) with 1/mu = 1/a + 1/w^2 (the erf(w r)/r interaction of two Gaussian charges)."""
    alpha, w = 0.6, 0.7
    mu = 1.0 / (1.0 / alpha + 1.0 / (w * w))
    ex = _isolated_gaussian_exchange(L, n, kmesh, kernels.TRUNC_ERF_LR, w, alpha)
    assert abs(ex + math.sqrt(mu / math.pi)) < 1e-11


# ----------------------------------------------------------------------------
# Madelung mode: the G + q = 0 value N_k Omega M_s of the Coulomb kernel
# ----------------------------------------------------------------------------

def test_madelung_constants_of_cubic_lattices():
    """Ewald Madelung constants of unit point charges in a neutralising background:
    simple cubic xi = 2.837297 / L; fcc and bcc 1.791747 and 1.791858 over the
    Wigner-Seitz radius (textbook values)."""
    assert abs(kernels.madelung(np.eye(3) * 7.3) * 7.3 - 2.837297479) < 1e-8
    fcc = np.array([[0, .5, .5], [.5, 0, .5], [.5, .5, 0]]) * 3.1
    bcc = np.array([[-.5, .5, .5], [.5, -.5, .5], [.5, .5, -.5]]) * 2.2
    for lat, ref in ((fcc, 1.791747), (bcc, 1.791858)):
        rws = (3.0 * abs(np.linalg.det(lat)) / (4.0 * math.pi)) ** (1.0 / 3.0)
        assert abs(kernels.madelung(lat) * rws - ref) < 2e-6


def test_madelung_mode_removes_the_image_term_of_an_s_gaussian():
    """With the G = 0 term set to Omega xi / L the single s-Gaussian's E_x loses its
    xi / 2L image term: -sqrt(a/pi) - pi / (2 a L^3) exactly."""
    L, alpha = 18.0, 0.6
    cell = W.cubic_cell(L, [(0.5, 0.5, 0.5)])
    basis = W.Basis(np.zeros(1, np.int32), np.zeros(1, np.int32), np.array([alpha]))
    prob = W.Problem("sgauss", cell, basis, (1, 1, 1), (60, 60, 60), 1, seed=0)
    C = np.ones((1, 1, 1), dtype=complex)
    ex = occrik.build(prob, C, want_k=False, madelung=True)["Ex"]
    assert abs(ex - (-math.sqrt(alpha / math.pi) - math.pi / (2 * alpha * L ** 3))) < 1e-10


def test_madelung_mode_kmesh_equals_gamma_supercell():
    """The k-mesh build uses the Born-von Karman supercell's constant, the Gamma build of
    that supercell its own: the per-cell energies agree (aliasing level)."""
    prob = W.small_problem(kmesh=(2, 1, 2), grid=(16, 16, 16), nocc=2, counts=(2, 1), amin=0.35, amax=0.9)
    C = W.random_coefficients(prob)
    e_k = occrik.build(prob, C, want_k=False, madelung=True)["Ex"]
    sc, Csc = _supercell(prob, C)
    e_sc = occrik.build(sc, Csc, want_k=False, madelung=True)["Ex"]
    assert abs(e_sc / prob.nk - e_k) < 1e-9 * abs(e_k)


def test_madelung_mode_keeps_long_plus_short_range_equal_to_coulomb(small):
    prob, C, res = small
    w = 0.45
    e_sr = occrik.build(prob, C, chi=res["chi"], want_k=False, kind=kernels.ERFC_SR, omega=w)["Ex"]
    e_lr = occrik.build(prob, C, chi=res["chi"], want_k=False, kind=kernels.ERF_LR, omega=w, madelung=True)["Ex"]
    e_co = occrik.build(prob, C, chi=res["chi"], want_k=False, kind=kernels.COULOMB, madelung=True)["Ex"]
    assert abs(e_sr + e_lr - e_co) < 1e-12 * abs(e_co)


# ----------------------------------------------------------------------------
# Conduction-band extension (Sec. II.D): K~ exact on occupied + selected bands
# ----------------------------------------------------------------------------

def test_conduction_band_extension_is_exact_on_the_selected_bands():
    """With nvir extra columns the exchange is still that of the occupied density, and
    K~ reproduces the conventional exchange on every selected band:
    K~ C_p = K_conv C_p and C_p^H K~ C_q = C_p^H K_conv C_q for p, q in occ + vir;
    E_x is the occupied-only one."""
    nocc, nvir = 2, 2
    prob = W.small_problem(kmesh=(2, 1, 1), grid=(10, 9, 8), nocc=nocc + nvir, counts=(2, 1, 1))
    C = W.random_coefficients(prob)                  # nocc + nvir orthonormal columns per k
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
    res = occrik.build(prob, C, chi=chi, nvir=nvir)
    occ_only = occrik.build(prob, C[:, :, :nocc], chi=chi)
    Kc = conventional.mo_k(prob, C[:, :, :nocc], chi)
    assert abs(res["Ex"] - occ_only["Ex"]) < 1e-13 * abs(occ_only["Ex"])
    KC = np.einsum("kmn,knp->kmp", res["K"], C)
    KcC = np.einsum("kmn,knp->kmp", Kc, C)
    assert np.max(np.abs(KC - KcC)) < 1e-11 * np.max(np.abs(KcC))
    assert np.max(np.abs(res["Kmi"] - KcC)) < 1e-11 * np.max(np.abs(KcC))
    blk = np.einsum("kmp,kmn,knq->kpq", np.conj(C), res["K"], C)
    blk_c = np.einsum("kmp,kmn,knq->kpq", np.conj(C), Kc, C)
    assert np.max(np.abs(blk - blk_c)) < 1e-11 * np.max(np.abs(blk_c))
    # without the extension the virtual rows of K~ are not the conventional ones
    KC0 = np.einsum("kmn,knp->kmp", occ_only["K"], C)
    assert np.max(np.abs(KC0[:, :, nocc:] - KcC[:, :, nocc:])) > 1e-4 * np.max(np.abs(KcC))
