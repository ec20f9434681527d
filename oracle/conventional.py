"""Conventional GPW exchange matrices (test infrastructure).

* MO-RI-K (paper Alg. 2, eqs. exxmo and mointerm2): for each output k2 and AO
  mu, the densities psi*_{i k1} chi_{mu k2} are fitted, their potentials
  V_{i k1, mu k2} formed, W_mu = sum_{k1, i} psi_{i k1} V_{i k1, mu k2}, and
  K_{nu mu}(k2) = -(dV/N_k) sum_r W_mu(r) chi*_{nu k2}(r)  (eq. aok with W).
* AO-RI-K (paper Alg. 1, eqs. aointerm, aointerm2, aok): psi~_{sigma k1} =
  sum_lambda P_{lambda sigma}(k1) chi_{lambda k1}, densities chi*_{sigma k1} chi_{mu k2},
  V~_mu = sum_{k1, sigma} psi~_{sigma k1} V_{sigma k1, mu k2}, K = -(dV/N_k) sum_r V~_mu chi*_nu.

Both give the full AO x AO exchange matrix on the same grid and with the same
normalisation as ``occrik``.  The occ-RI-K identities K C = K_{mu j},
C^H K C = K_ij and the equal exchange energy (paper Sec. II.D) are checked
against them.
"""
import numpy as np

from .occrik import Geometry, pair_potentials


def mo_k(prob, C, chi, out_k=None, kind=None, omega=None, nyquist="fftfreq"):
    geo = Geometry(prob.cell, prob.kmesh, prob.grid)
    kind = prob.kernel if kind is None else kind
    omega = prob.omega if omega is None else omega
    out_k = list(range(geo.nk)) if out_k is None else list(out_k)
    psi = np.einsum("kmi,kmn->kin", C, chi)                       # eq. occmo
    nao = chi.shape[1]
    K = np.zeros((len(out_k), nao, nao), dtype=np.complex128)
    for a, k2 in enumerate(out_k):
        W = np.zeros((nao, geo.ng), dtype=np.complex128)
        for mu in range(nao):
            for k1 in range(geo.nk):
                rho = np.conj(psi[k1]) * chi[k2, mu][None, :]
                V, _ = pair_potentials(geo, rho, k2, k1, kind, omega, nyquist)
                W[mu] += np.sum(psi[k1] * V, axis=0)
        # K[nu, mu] = -(dV/N_k) sum_r W_mu chi*_nu
        K[a] = -(geo.dv / geo.nk) * (np.conj(chi[k2]) @ W.T)
    return K


def ao_k(prob, C, chi, out_k=None, kind=None, omega=None, nyquist="fftfreq"):
    geo = Geometry(prob.cell, prob.kmesh, prob.grid)
    kind = prob.kernel if kind is None else kind
    omega = prob.omega if omega is None else omega
    out_k = list(range(geo.nk)) if out_k is None else list(out_k)
    P = np.einsum("kli,ksi->kls", C, np.conj(C))                  # P_{lambda sigma}
    psit = np.einsum("kls,kln->ksn", P, chi)                       # eq. aointerm
    nao = chi.shape[1]
    K = np.zeros((len(out_k), nao, nao), dtype=np.complex128)
    for a, k2 in enumerate(out_k):
        Vt = np.zeros((nao, geo.ng), dtype=np.complex128)
        for mu in range(nao):
            for k1 in range(geo.nk):
                rho = np.conj(chi[k1]) * chi[k2, mu][None, :]        # all sigma at once
                V, _ = pair_potentials(geo, rho, k2, k1, kind, omega, nyquist)
                Vt[mu] += np.sum(psit[k1] * V, axis=0)               # eq. aointerm2
        K[a] = -(geo.dv / geo.nk) * (np.conj(chi[k2]) @ Vt.T)       # eq. aok
    return K
