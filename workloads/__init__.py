"""Seeded synthetic inputs for the occ-RI-K exchange build.

This module generates *inputs only*: the periodic cell, the uncontracted
cartesian Gaussian basis, the Gamma-centred k-mesh, the real-space grid and the
occupied-orbital coefficients C_occ(k).  It holds none of the exchange method's
arithmetic (no collocation, no FFT, no Coulomb kernel, no contraction).  Both
the CPU oracle (``oracle/``) and the GPU library's tests draw their inputs from
here, so that the two sides see identical numbers while sharing no method code.

Conventions fixed by the inputs (stated once, honoured by both consumers):

* lengths in bohr; lattice rows a_1, a_2, a_3; atoms in fractional coordinates;
* k-mesh: Gamma-centred, k = sum_d (kappa_d / M_d) b_d with kappa_d in [0, M_d),
  row-major over (kappa_1, kappa_2, kappa_3) (kappa_3 fastest);
* grid: r_n = sum_d (n_d / N_d) a_d, row-major over (n_1, n_2, n_3);
* shells: uncontracted cartesian, ordered per atom, then by l, then by exponent
  (ascending); components inside a shell in lexicographic order
  (x^l first: xx, xy, xz, yy, yz, zz for l = 2);
* each cartesian component is normalised as an isolated function:
  N = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!);
* C_occ(k) = X_k (X_k^H S_k X_k)^(-1/2) with Re X, Im X iid N(0,1) drawn from
  ``numpy.random.default_rng(seed)`` in k order (real block, then imaginary
  block), and S_k the analytic lattice-summed overlap.  Orbitals are therefore
  orthonormal over one unit cell (the per-cell convention of the Bloch sum with
  its 1/sqrt(N_k) dropped, paper Sec. II.A).

The workloads mirror the paper's timing system (a two-atom diamond cell,
Sec. IV.A) and its largest production run (350 basis functions, 16 electrons,
6x6x6 k-mesh, Sec. III); the paper's own basis sets and pseudopotentials are not
available, so geometric even-tempered exponent ladders stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Sequence, Tuple


import numpy as np

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903

KERNEL_COULOMB = 0
KERNEL_ERF_LR = 1
KERNEL_ERFC_SR = 2
KERNEL_TRUNC_COULOMB = 3
KERNEL_TRUNC_ERF_LR = 4


@dataclass
class Cell:
    lattice: np.ndarray          # (3, 3) rows a_1..a_3, bohr
    atoms_frac: np.ndarray       # (natm, 3) fractional coordinates

    @property
    def natm(self) -> int:
        return int(self.atoms_frac.shape[0])


@dataclass
class Basis:
    shell_atom: np.ndarray       # (nshell,) int32
    shell_l: np.ndarray          # (nshell,) int32
    shell_exp: np.ndarray        # (nshell,) float64

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nao(self) -> int:
        return int(sum((l + 1) * (l + 2) // 2 for l in self.shell_l))


@dataclass
class Problem:
    name: str
    cell: Cell
    basis: Basis
    kmesh: Tuple[int, int, int]
    grid: Tuple[int, int, int]
    nocc: int
    kernel: int = KERNEL_COULOMB
    omega: float = 0.0
    seed: int = 0
    lattice_tol: float = 1e-12

    @property
    def nk(self) -> int:
        return int(np.prod(self.kmesh))

    @property
    def ng(self) -> int:
        return int(np.prod(self.grid))

    @property
    def nao(self) -> int:
        return self.basis.nao


def cart_components(l: int) -> List[Tuple[int, int, int]]:
    """Cartesian exponent triples of a shell, lexicographic (x^l first)."""
    out = []
    for lx in range(l, -1, -1):
        for ly in range(l - lx, -1, -1):
            out.append((lx, ly, l - lx - ly))
    return out


def _dfact(n: int) -> float:
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


def cart_norm(alpha: float, lx: int, ly: int, lz: int) -> float:
    l = lx + ly + lz
    return ((2 * alpha / np.pi) ** 0.75 * (4 * alpha) ** (l / 2.0)
            / np.sqrt(_dfact(2 * lx - 1) * _dfact(2 * ly - 1) * _dfact(2 * lz - 1)))


# ----------------------------------------------------------------------------
# cells
# ----------------------------------------------------------------------------

def fcc_lattice(a_bohr: float) -> np.ndarray:
    h = 0.5 * a_bohr
    return np.array([[0.0, h, h], [h, 0.0, h], [h, h, 0.0]])


def bcc_lattice(a_bohr: float) -> np.ndarray:
    h = 0.5 * a_bohr
    return np.array([[-h, h, h], [h, -h, h], [h, h, -h]])


def diamond_cell() -> Cell:
    """Two-atom fcc diamond cell, a = 3.57 Angstrom (paper Sec. IV.A timing system)."""
    a = 3.57 * BOHR_PER_ANGSTROM
    return Cell(fcc_lattice(a), np.array([[0.0, 0.0, 0.0], [0.25, 0.25, 0.25]]))


def cubic_cell(L: float, atoms_frac=((0.0, 0.0, 0.0),)) -> Cell:
    return Cell(np.eye(3) * L, np.array(atoms_frac, dtype=float))


# ----------------------------------------------------------------------------
# bases
# ----------------------------------------------------------------------------

def geometric_exponents(n: int, amin: float, amax: float) -> np.ndarray:
    if n == 1:
        return np.array([np.sqrt(amin * amax)])
    return amin * (amax / amin) ** (np.arange(n) / (n - 1.0))


def even_tempered_basis(natm: int, counts: Sequence[int], amin: float, amax: float,
                        per_atom_counts: Sequence[Sequence[int]] | None = None) -> Basis:
    """Per atom: for l = 0.. len(counts)-1, counts[l] shells with geometric exponents."""
    sa, sl, se = [], [], []
    for a in range(natm):
        cts = counts if per_atom_counts is None else per_atom_counts[a]
        for l, n in enumerate(cts):
            if n <= 0:
                continue
            for e in geometric_exponents(n, amin, amax):
                sa.append(a)
                sl.append(l)
                se.append(e)
    return Basis(np.array(sa, dtype=np.int32), np.array(sl, dtype=np.int32),
                 np.array(se, dtype=np.float64))


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

def make_problem(name: str) -> Problem:
    """Named workloads.

    tiny     2-atom diamond, s4 p3 per atom (26 AO), alpha in [0.15, 12], 4 occ,
             2x2x2 k, 24^3 grid, Coulomb.  (``tiny14``: the literal s5 p3 recipe, 28 AO.)
    prec     s8 p8 d3 per atom (100 AO), alpha in [0.08, 30], 4 occ, 3x3x3 k, 36^3.
    paper    s20 p15 d10 f5 per atom (350 AO), alpha in [0.05, 50], 8 occ, 6x6x6 k, 48^3.
    diff     s10 p10 d5 f3 per atom (200 AO), alpha in [0.05, 50], 8 occ, 4x4x4 k, 40^3,
             long-range erf kernel with omega = 0.3.
    """
    cell = diamond_cell()
    if name == "tiny":
        return Problem(name, cell, even_tempered_basis(2, [4, 3], 0.15, 12.0), (2, 2, 2), (24, 24, 24), 4, seed=11)
    if name == "tiny14":
        return Problem(name, cell, even_tempered_basis(2, [5, 3], 0.15, 12.0), (2, 2, 2), (24, 24, 24), 4, seed=12)
    if name == "prec":
        return Problem(name, cell, even_tempered_basis(2, [8, 8, 3], 0.08, 30.0), (3, 3, 3), (36, 36, 36), 4, seed=13)
    if name == "paper":
        return Problem(name, cell, even_tempered_basis(2, [20, 15, 10, 5], 0.05, 50.0), (6, 6, 6), (48, 48, 48), 8, seed=14)
    if name == "diff":
        return Problem(name, cell, even_tempered_basis(2, [10, 10, 5, 3], 0.05, 50.0), (4, 4, 4), (40, 40, 40), 8,
                       kernel=KERNEL_ERF_LR, omega=0.3, seed=15)
    raise KeyError(name)


def small_problem(kmesh=(2, 1, 3), grid=(12, 10, 9), nocc=3, counts=(2, 1, 1), amin=0.3, amax=3.0,
                  kernel=KERNEL_COULOMB, omega=0.0, seed=5, cell: Cell | None = None,
                  lattice_tol: float = 1e-12) -> Problem:
    """A small, deliberately ragged problem for fast tests (odd grid sizes, uneven k-mesh)."""
    cell = diamond_cell() if cell is None else cell
    basis = even_tempered_basis(cell.natm, list(counts), amin, amax)
    return Problem("small", cell, basis, tuple(kmesh), tuple(grid), nocc, kernel=kernel, omega=omega,
                   seed=seed, lattice_tol=lattice_tol)


def batch_problems(n: int = 64, seed: int = 1000) -> List[Problem]:
    """Ragged batch of cells: fcc/bcc/rocksalt, a in [3, 6] Angstrom, 1-4 atoms,
    N_AO in [50, 350] with an s:p:d:f ~ 4:3:2:1 shell fill, N_occ in 4..8,
    k-meshes M^3 with M in {2,3,4}, grids N^3 with N in {24,30,32,36,40,48}."""
    out = []
    for c in range(n):
        rng = np.random.default_rng(seed + c)
        kind = ["fcc", "bcc", "rocksalt"][int(rng.integers(3))]
        a = float(rng.uniform(3.0, 6.0)) * BOHR_PER_ANGSTROM
        lat = bcc_lattice(a) if kind == "bcc" else fcc_lattice(a)
        natm = int(rng.integers(1, 5))
        sites = [[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]] if kind == "rocksalt" else \
            ([[0.0, 0.0, 0.0], [0.25, 0.25, 0.25], [0.5, 0.5, 0.5], [0.75, 0.75, 0.75]] if kind == "fcc"
             else [[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
        atoms = sites[:natm]
        while len(atoms) < natm:
            f = rng.uniform(0.0, 1.0, 3)
            ok = True
            for g in atoms:
                d = f - np.array(g)
                d -= np.round(d)
                if np.linalg.norm(d @ lat) < 1.5:
                    ok = False
            if ok:
                atoms.append(list(f))
        nao_target = int(rng.integers(50, 351))
        per_atom = [nao_target // natm + (1 if i < nao_target % natm else 0) for i in range(natm)]
        counts = []
        for t in per_atom:
            cts = [0, 0, 0, 0]
            tot = 0
            cyc = [0, 0, 0, 0, 1, 1, 1, 2, 2, 3]      # 4 s : 3 p : 2 d : 1 f
            i = 0
            while True:
                l = cyc[i % len(cyc)]
                w = (l + 1) * (l + 2) // 2
                if tot + w > t:
                    break
                cts[l] += 1
                tot += w
                i += 1
            cts[0] += t - tot                          # top up with s shells
            counts.append(cts)
        basis = even_tempered_basis(natm, [0], 0.1, 30.0, per_atom_counts=counts)
        m = int(rng.choice([2, 3, 4]))
        g = int(rng.choice([24, 30, 32, 36, 40, 48]))
        nocc = int(rng.integers(4, 9))
        out.append(Problem(f"batch{c}", Cell(lat, np.array(atoms, dtype=float)), basis, (m, m, m), (g, g, g),
                           nocc, seed=seed + 7919 * (c + 1)))
    return out


def batch_parity_problems() -> List[Problem]:
    """Eight cells of the ragged batch (``batch_problems``) for parity against the FP64
    oracle: their cells, bases (51-350 AOs) and occupied counts (4-8), with the k-mesh
    and grid capped so that the oracle builds all eight in a few minutes.  Grids: the
    compiled sizes 24^3, 30^3 and 32^3 and the run-time sizes 27 x 25 x 20 and 20^3;
    k-meshes 2^3 and one 3^3."""
    full = batch_problems()
    picks = [(57, None, None), (8, None, None), (34, None, None), (55, None, None), (44, None, None),
             (51, (27, 25, 20), None), (16, (20, 20, 20), None), (43, None, (2, 2, 2))]
    out = []
    for idx, grid, kmesh in picks:
        p = full[idx]
        if grid is not None:
            p = replace(p, grid=grid)
        if kmesh is not None:
            p = replace(p, kmesh=kmesh)
        out.append(p)
    return out


# ----------------------------------------------------------------------------
# k-points and the analytic overlap (used only to orthonormalise C_occ)
# ----------------------------------------------------------------------------

def kpoints_frac(kmesh) -> np.ndarray:
    M = np.array(kmesh)
    idx = np.stack(np.meshgrid(*[np.arange(m) for m in kmesh], indexing="ij"), -1).reshape(-1, 3)
    return idx / M


def reciprocal(lattice: np.ndarray) -> np.ndarray:
    return 2.0 * np.pi * np.linalg.inv(lattice).T


def _os_1d(la: int, lb: int, PA: np.ndarray, PB: np.ndarray, p: float) -> np.ndarray:
    """Obara-Saika 1D overlap table S[a, b] / S[0, 0] for arrays of geometries."""
    S = np.zeros((la + 1, lb + 1) + PA.shape)
    S[0, 0] = 1.0
    inv2p = 0.5 / p
    for a in range(la + 1):
        for b in range(lb + 1):
            if a == 0 and b == 0:
                continue
            if a > 0:
                v = PA * S[a - 1, b]
                if a > 1:
                    v = v + inv2p * (a - 1) * S[a - 2, b]
                if b > 0:
                    v = v + inv2p * b * S[a - 1, b - 1]
            else:
                v = PB * S[a, b - 1]
                if b > 1:
                    v = v + inv2p * (b - 1) * S[a, b - 2]
            S[a, b] = v
    return S


def overlap_k(prob: Problem) -> np.ndarray:
    """S_k[mu, nu] = sum_T exp(i k.T) <phi_mu(r - R_mu) | phi_nu(r - R_nu - T)>, analytic."""
    cell, basis = prob.cell, prob.basis
    lat = cell.lattice
    kf = kpoints_frac(prob.kmesh)
    centers = cell.atoms_frac @ lat
    offs = []
    o = 0
    for l in basis.shell_l:
        offs.append(o)
        o += (l + 1) * (l + 2) // 2
    nao = o
    S = np.zeros((prob.nk, nao, nao), dtype=np.complex128)
    amin = float(np.min(basis.shell_exp))
    # image lattice generous enough for the most diffuse pair
    pmin = amin / 2.0
    rmax = np.sqrt(50.0 / pmin) + np.max(np.linalg.norm(lat, axis=1)) * 2
    inv = np.linalg.inv(lat)
    nmax = [int(np.ceil(rmax * np.linalg.norm(inv[:, d]))) + 1 for d in range(3)]
    tr_all = np.stack(np.meshgrid(*[np.arange(-n, n + 1) for n in nmax], indexing="ij"), -1).reshape(-1, 3)
    # per atom pair: images sorted by distance, so every shell pair keeps a prefix
    pair_cache = {}
    for ia in range(cell.natm):
        for ib in range(cell.natm):
            d = centers[ia][None, :] - (centers[ib][None, :] + tr_all @ lat)
            d2 = np.sum(d * d, axis=1)
            order = np.argsort(d2, kind="stable")
            tri = tr_all[order]
            arg = 2.0 * np.pi * (kf @ tri.T)
            pair_cache[(ia, ib)] = (tri @ lat, d2[order], np.cos(arg), np.sin(arg))
    for si in range(basis.nshell):
        la, a = int(basis.shell_l[si]), float(basis.shell_exp[si])
        ia = int(basis.shell_atom[si])
        A = centers[ia]
        ca = cart_components(la)
        na_ = [cart_norm(a, *c) for c in ca]
        for sj in range(basis.nshell):
            lb, b = int(basis.shell_l[sj]), float(basis.shell_exp[sj])
            ib = int(basis.shell_atom[sj])
            B0 = centers[ib]
            cb = cart_components(lb)
            p = a + b
            mu = a * b / p
            T_s, d2_s, cos_s, sin_s = pair_cache[(ia, ib)]
            n = int(np.searchsorted(d2_s, (45.0 + 2.0 * (la + lb)) / mu, side="left"))
            if n == 0:
                continue
            T = T_s[:n]
            Bs = B0[None, :] + T
            P = (a * A[None, :] + b * Bs) / p
            PA = P - A[None, :]
            PB = P - Bs
            pref = (np.pi / p) ** 1.5 * np.exp(-mu * d2_s[:n])
            tabs = [_os_1d(la, lb, PA[:, x], PB[:, x], p) for x in range(3)]
            blk = np.empty((len(ca) * len(cb), n))
            for iaa, (ax, ay, az) in enumerate(ca):
                for ibb, (bx, by, bz) in enumerate(cb):
                    nb = cart_norm(b, bx, by, bz)
                    blk[iaa * len(cb) + ibb] = (na_[iaa] * nb) * pref * tabs[0][ax, bx] * tabs[1][ay, by] * tabs[2][az, bz]
            re = cos_s[:, :n] @ blk.T
            im = sin_s[:, :n] @ blk.T
            S[:, offs[si]:offs[si] + len(ca), offs[sj]:offs[sj] + len(cb)] = (re + 1j * im).reshape(
                prob.nk, len(ca), len(cb))
    return S


def random_coefficients(prob: Problem, orthonormalise: bool = True) -> np.ndarray:
    """C_occ[k, mu, i] complex128, seeded; S_k-orthonormal columns when requested."""
    rng = np.random.default_rng(prob.seed)
    nk, nao, nocc = prob.nk, prob.nao, prob.nocc
    X = np.empty((nk, nao, nocc), dtype=np.complex128)
    for k in range(nk):
        re = rng.standard_normal((nao, nocc))
        im = rng.standard_normal((nao, nocc))
        X[k] = re + 1j * im
    if not orthonormalise:
        return X
    S = overlap_k(prob)
    C = np.empty_like(X)
    for k in range(nk):
        M = X[k].conj().T @ S[k] @ X[k]
        M = 0.5 * (M + M.conj().T)
        w, U = np.linalg.eigh(M)
        C[k] = X[k] @ (U * (1.0 / np.sqrt(w))) @ U.conj().T
    return C


def with_kernel(prob: Problem, kernel: int, omega: float) -> Problem:
    return replace(prob, kernel=kernel, omega=omega)
