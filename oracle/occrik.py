"""occ-RI-K exchange build, written out from the paper in FP64 (test infrastructure).

Notation follows Alg. 3 of the paper: the output k-point is k2 with occupied
index j, the summed k-point is k1 with occupied index i.

* eq. occmo:          psi_{i k}(r) = sum_mu C_{mu i}(k) chi_{mu k}(r)
* eqs. aodf, Vrao, VGao: the pair density rho(r) = psi*_{i k1}(r) psi_{j k2}(r) carries
  momentum q = k2 - k1; its plane-wave coefficients are
  Z^G = (1/Omega) int rho exp(-i(G+q).r) dr  ->  (1/N_g) DFT[rho exp(-i q.r)](G),
  the potential is V(r) = sum_G f(|G+q|) Z^G exp(i(G+q).r), with the G+q = 0 term
  replaced by the kernel's chi constant.
* eq. occrikinterm:   W_{j k2}(r) = sum_{k1, i} psi_{i k1}(r) V_{i k1, j k2}(r)
* contraction (the second equation labelled occrik):
  K_{nu j}(k2) = -(dV / N_k) sum_r W_{j k2}(r) chi*_{nu k2}(r).
  The paper writes a bare sum over r; dV = Omega / N_g turns it into the cell
  integral and 1/N_k is the Bloch normalisation the orbitals here omit.  With it,
  E = (1/2N_k) sum_k Re tr(C^H K C) is the paper's E_K / N_k (Sec. II.A), the
  exchange energy per cell and per spin channel.
* eq. occrikop: the occupied block K_ij = C^H K_{mu j} and the assembled matrix
  K~ = K_mu (K_ij)^-1 K_mu^H, computed through the Cholesky factor of -K_ij.

Pair momenta are never wrapped: q = k2 - k1 from fractional k-points in [0, 1).
FFT index order is numpy's (the even-N Nyquist bin is -N/2).  The DFTs are
scipy.fft's (pocketfft, the same unnormalised definition as numpy.fft), run over
the stack of pair densities with ``FFT_WORKERS`` threads: the host's cores, or
OMP_NUM_THREADS when that is set.  ``nyquist`` =
"symmetric" replaces f on the Nyquist planes by the mean of f at G_m + q and at
the mirror index whose Nyquist components are +N/2 (the only change between the
two modes).
"""
import os

import numpy as np
import scipy.fft

from . import collocation
from . import kernels
from . import lattice as lat_mod


FFT_WORKERS = max(1, int(os.environ.get("OMP_NUM_THREADS") or 0) or (os.cpu_count() or 1))


def _dft3(u):
    """Unnormalised forward DFT over the last three axes."""
    return scipy.fft.fftn(u, axes=(-3, -2, -1), workers=FFT_WORKERS)


def _idft3(u):
    """Inverse DFT over the last three axes, with the 1/N_g of numpy's convention."""
    return scipy.fft.ifftn(u, axes=(-3, -2, -1), workers=FFT_WORKERS)


class Geometry:
    """Everything the pair loop needs that depends only on cell, mesh and grid."""

    def __init__(self, cell, kmesh, grid, madelung=False):
        self.lattice = np.asarray(cell.lattice, dtype=float)
        self.kmesh = tuple(int(x) for x in kmesh)
        self.grid = tuple(int(x) for x in grid)
        self.omega_cell = lat_mod.volume(self.lattice)
        self.recip = lat_mod.reciprocal_vectors(self.lattice)
        self.r = lat_mod.grid_points(self.lattice, self.grid)
        self.ng = self.r.shape[0]
        self.dv = self.omega_cell / self.ng
        self.kfrac = lat_mod.kpoints_fractional(self.kmesh)
        self.kcart = self.kfrac @ self.recip
        self.nk = self.kfrac.shape[0]
        self.miller = lat_mod.miller_grid(self.grid)
        self.rcut = kernels.truncation_radius(self.nk, self.omega_cell)
        # Madelung mode: G + q = 0 value of the Coulomb kernel, N_k Omega M_s of the
        # Born-von Karman supercell (its rows M_d a_d)
        self.g0_coulomb = None
        if madelung:
            sup = np.asarray(self.kmesh, dtype=float)[:, None] * self.lattice
            self.g0_coulomb = self.nk * self.omega_cell * kernels.madelung(sup)

    def momentum_sq(self, q_frac, mirror=False):
        """|G_m + q|^2 over the DFT grid; ``mirror`` flips Nyquist components to +N/2."""
        m = self.miller.astype(float)
        if mirror:
            m = m.copy()
            for d, n in enumerate(self.grid):
                if n % 2 == 0:
                    m[m[:, d] == -(n // 2), d] = n // 2
        g = (m + q_frac[None, :]) @ self.recip
        return np.sum(g * g, axis=1)

    def kernel_on_grid(self, k2, k1, kind, omega, nyquist="fftfreq", derivative=False):
        q = self.kfrac[k2] - self.kfrac[k1]
        if derivative:
            def fn(x2):
                return kernels.kernel_domega(x2, kind, omega, self.rcut)
        else:
            def fn(x2):
                return kernels.kernel_values(x2, kind, omega, self.rcut)
        v = fn(self.momentum_sq(q))
        if nyquist == "symmetric":
            v = 0.5 * (v + fn(self.momentum_sq(q, mirror=True)))
        elif nyquist != "fftfreq":
            raise ValueError(nyquist)
        if self.g0_coulomb is not None and k2 == k1 and kind in (kernels.COULOMB, kernels.ERF_LR):
            # G = 0 is grid index 0; q = 0 exactly for k2 == k1
            if derivative:
                v[0] = 0.0 if kind == kernels.COULOMB else 2.0 * np.pi / omega ** 3
            else:
                v[0] = self.g0_coulomb - (0.0 if kind == kernels.COULOMB else np.pi / (omega * omega))
        return v.reshape(self.grid)


def occupied_orbitals(chi, C):
    """eq. occmo: psi[k, i, n] = sum_mu C[k, mu, i] chi[k, mu, n]."""
    return np.einsum("kmi,kmn->kin", C, chi)


def pair_potentials(geo, rho, k2, k1, kind, omega, nyquist="fftfreq", want_parseval=False):
    """Potentials of a stack of pair densities rho[..., n] with momentum q = k2 - k1.

    Returns V[..., n] and, when requested, the per-density sums
    sum_m f |DFT[rho e^{-iq.r}]_m|^2 (used by the Parseval form of the energy).
    """
    qc = geo.kcart[k2] - geo.kcart[k1]
    ph = np.exp(-1j * (geo.r @ qc))                          # e^{-i q.r}
    shape = rho.shape[:-1] + geo.grid
    u = (rho * ph).reshape(shape)
    uhat = _dft3(u)                                          # unnormalised DFT
    v = geo.kernel_on_grid(k2, k1, kind, omega, nyquist)
    Z = uhat / geo.ng                                        # Z^G
    Vt = _idft3(v * Z) * geo.ng                              # sum_G V^G e^{iG.r}
    V = Vt.reshape(rho.shape) * np.conj(ph)                  # times e^{iq.r}
    if not want_parseval:
        return V, None
    return V, np.sum(v * np.abs(uhat) ** 2, axis=(-3, -2, -1))


def exchange_w(geo, psi, out_k, kind, omega, nyquist="fftfreq", parseval=False, domega=False, k1_subset=None,
               nsum=None):
    """Alg. 3 loops: W[k2][j] = sum_{k1, i} psi_{i k1} V_{i k1, j k2} for k2 in out_k.

    The sum runs over the first ``nsum`` orbitals of psi (the occupied ones; all by
    default); W is formed for every orbital j of psi at k2, which with extra columns
    is the conduction-band extension of Sec. II.D (exchange still built from the
    occupied density).  Also returns the Parseval partial sums sum f |u^|^2 (and
    sum df/dw |u^|^2) over the occupied pairs, when requested.  ``k1_subset``
    restricts the summed k-points (a partial sum, used only to time a bounded
    sample of the loops).
    """
    nout = psi.shape[1]
    nsum = nout if nsum is None else nsum
    W = np.zeros((len(out_k), nout, geo.ng), dtype=np.complex128)
    ps = 0.0
    pd = 0.0
    k1_list = range(geo.nk) if k1_subset is None else list(k1_subset)
    for a, k2 in enumerate(out_k):
        for j in range(nout):
            occ_pair = j < nsum
            for k1 in k1_list:
                rho = np.conj(psi[k1, :nsum]) * psi[k2, j][None, :]    # all summed i at once
                V, s = pair_potentials(geo, rho, k2, k1, kind, omega, nyquist,
                                       want_parseval=occ_pair and (parseval or domega))
                W[a, j] += np.sum(psi[k1, :nsum] * V, axis=0)
                if parseval and occ_pair:
                    ps += float(np.sum(s))
                if domega and occ_pair:
                    qc = geo.kcart[k2] - geo.kcart[k1]
                    ph = np.exp(-1j * (geo.r @ qc))
                    uhat = _dft3((rho * ph).reshape((nsum,) + geo.grid))
                    dv = geo.kernel_on_grid(k2, k1, kind, omega, nyquist, derivative=True)
                    pd += float(np.sum(dv * np.abs(uhat) ** 2))
    return W, ps, pd


def contract(geo, chi_out, W):
    """K_{nu j}(k2) = -(dV/N_k) sum_r chi*_{nu k2}(r) W_{j k2}(r); shape (nout, nao, nocc)."""
    return -(geo.dv / geo.nk) * np.einsum("kmn,kjn->kmj", np.conj(chi_out), W)


def occupied_block(C_out, Kmi):
    """K_ij(k) = sum_mu C*_{mu i}(k) K_{mu j}(k)."""
    return np.einsum("kmi,kmj->kij", np.conj(C_out), Kmi)


def exchange_energy_terms(Kij, nk, nocc=None):
    """Per-k contributions Re tr K_ij(k) / (2 N_k) over the occupied block (the first
    ``nocc`` orbitals; all by default); their sum over all k is E_x."""
    n = Kij.shape[1] if nocc is None else nocc
    return np.real(np.einsum("kii->k", Kij[:, :n, :n])) / (2.0 * nk)


def assemble(Kmi, Kij):
    """K~(k) = K_mu (K_ij)^-1 K_mu^H via L L^H = -K_ij, xi = K_mu L^-H, K~ = -xi xi^H.

    Raises numpy.linalg.LinAlgError when -K_ij is not positive definite.
    """
    out = np.empty((Kmi.shape[0], Kmi.shape[1], Kmi.shape[1]), dtype=np.complex128)
    for k in range(Kmi.shape[0]):
        A = -0.5 * (Kij[k] + Kij[k].conj().T)
        L = np.linalg.cholesky(A)
        xi_h = np.linalg.solve(L, Kmi[k].conj().T)                # L^-1 K^H = xi^H
        out[k] = -(xi_h.conj().T @ xi_h)
    return out


def assemble_projector(Kmi, Kij, S, C):
    """Paper eq. occrikop written with projectors: K_P = K_mu (SC)^H + (SC) K_mu^H - (SC) K_ij (SC)^H.

    Pinned by the identities K_P C = K_mu and C^H K_P C = K_ij (which hold when
    C^H S C = 1) and, with as many orbitals as AOs, by equality with the
    conventional AO-RI-K matrix (Alg. 1).  It is not on the GPU path.
    """
    out = np.empty((Kmi.shape[0], Kmi.shape[1], Kmi.shape[1]), dtype=np.complex128)
    for k in range(Kmi.shape[0]):
        SC = S[k] @ C[k]
        out[k] = Kmi[k] @ SC.conj().T + SC @ Kmi[k].conj().T - SC @ Kij[k] @ SC.conj().T
    return out


def build(prob, C, chi=None, out_k=None, nyquist="fftfreq", want_k=True, parseval=False, domega=False,
          kind=None, omega=None, madelung=False, nvir=0):
    """The whole occ-RI-K build for ``prob`` with coefficients C[k, mu, p].

    The last ``nvir`` columns of C are conduction bands treated exactly (Sec. II.D):
    the exchange is built from the occupied columns only, K_{mu p} and the block
    K_pq cover every column, and K~ = K_mu K_pq^-1 K_mu^H.  Returns a dict with chi
    (if computed here), psi, W, Kmi, Kij, ex_terms, Ex (the sum of ex_terms,
    complete only when out_k covers every k-point), K (assembled, when ``want_k``),
    and Parseval / d omega sums when requested.
    """
    geo = Geometry(prob.cell, prob.kmesh, prob.grid, madelung=madelung)
    kind = prob.kernel if kind is None else kind
    omega = prob.omega if omega is None else omega
    if chi is None:
        chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
    out_k = list(range(geo.nk)) if out_k is None else list(out_k)
    nocc = C.shape[2] - nvir
    psi = occupied_orbitals(chi, C)
    W, ps, pd = exchange_w(geo, psi, out_k, kind, omega, nyquist, parseval, domega, nsum=nocc)
    Kmi = contract(geo, chi[out_k], W)
    Kij = occupied_block(C[out_k], Kmi)
    terms = exchange_energy_terms(Kij, geo.nk, nocc)
    res = dict(chi=chi, psi=psi, W=W, Kmi=Kmi, Kij=Kij, ex_terms=terms, Ex=float(np.sum(terms)), out_k=out_k)
    if want_k:
        res["K"] = assemble(Kmi, Kij)
    scale = -geo.omega_cell / (2.0 * geo.nk ** 2 * geo.ng ** 2)
    if parseval:
        res["Ex_parseval"] = scale * ps
    if domega:
        res["dEx_domega"] = scale * pd
    return res


def energy_gradient_C(Kmi, nk):
    """d E_x / d Re C + i d E_x / d Im C = (2 / N_k) K_mu i (E_x = E_K / N_k, Sec. II.A)."""
    return (2.0 / nk) * Kmi
