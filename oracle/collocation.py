"""Bloch sums of cartesian Gaussians on the real-space grid (paper Sec. II.A).

Test infrastructure: see the package docstring.

chi_{mu k}(r_n) = sum_T exp(i k.T) phi_mu(r_n - R_mu - T)

is the paper's Bloch atomic orbital with its 1/sqrt(N_k) dropped, so orbitals
built from it are normalised over one unit cell.  phi_mu = N x^a y^b z^c
exp(-alpha r^2) with each cartesian component normalised as an isolated
function.  The lattice sum keeps every image T whose centre R_mu + T lies within
rho + r_s of the cell centre c = (a_1 + a_2 + a_3)/2, where rho is the cell's
circumradius about c and r_s solves N_s r^l exp(-alpha r^2) = tol beyond the
radial maximum (N_s = (2 alpha/pi)^(3/4) (4 alpha)^(l/2), the largest
component norm of the shell).  No grid point can then be within r_s of an
omitted image, so every omitted term is below tol in magnitude.
"""
import numpy as np

from . import lattice as lat_mod


def cartesian_powers(l):
    """(a, b, c) with a + b + c = l, lexicographic with x^l first."""
    return [(a, b, l - a - b) for a in range(l, -1, -1) for b in range(l - a, -1, -1)]


def _double_factorial(n):
    out = 1
    while n > 1:
        out *= n
        n -= 2
    return out


def component_norm(alpha, a, b, c):
    l = a + b + c
    return ((2.0 * alpha / np.pi) ** 0.75 * (4.0 * alpha) ** (0.5 * l)
            / np.sqrt(_double_factorial(2 * a - 1) * _double_factorial(2 * b - 1) * _double_factorial(2 * c - 1)))


def shell_extent(alpha, l, tol):
    """Largest r with N_s r^l exp(-alpha r^2) >= tol (radius beyond which the shell is below tol)."""
    ln_n = 0.75 * np.log(2.0 * alpha / np.pi) + 0.5 * l * np.log(4.0 * alpha)
    ln_tol = np.log(tol)

    def g(r):
        return ln_n + (l * np.log(r) if l > 0 else 0.0) - alpha * r * r - ln_tol

    lo = np.sqrt(l / (2.0 * alpha)) if l > 0 else 0.0
    if l > 0 and g(lo) < 0.0:
        return 0.0
    if l == 0 and ln_n - ln_tol < 0.0:
        return 0.0
    hi = max(lo, 1.0)
    while g(hi) > 0.0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return hi


def cell_center_and_radius(lattice):
    c = 0.5 * lattice.sum(axis=0)
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=float) @ lattice
    return c, float(np.max(np.linalg.norm(corners - c, axis=1)))


def shell_images(lattice, center, alpha, l, tol):
    """Integer image triples t (T = t @ lattice) kept by the truncation rule."""
    c, rho = cell_center_and_radius(lattice)
    rs = shell_extent(alpha, l, tol)
    reach = rho + rs
    bound = reach + np.linalg.norm(center - c)
    inv = np.linalg.inv(lattice)
    nmax = [int(np.ceil(bound * np.linalg.norm(inv[:, d]))) + 1 for d in range(3)]
    t = np.stack(np.meshgrid(*[np.arange(-n, n + 1) for n in nmax], indexing="ij"), -1).reshape(-1, 3)
    d = center[None, :] + t @ lattice - c[None, :]
    keep = np.sum(d * d, axis=1) <= reach * reach
    return t[keep]


def collocate(cell, basis, kmesh, grid, tol=1e-12, kpoint_indices=None, chunk=8192):
    """chi[k, mu, n] (complex128) for the requested k-points (all by default)."""
    lattice = cell.lattice
    kf = lat_mod.kpoints_fractional(kmesh)
    if kpoint_indices is not None:
        kf = kf[np.asarray(kpoint_indices)]
    r = lat_mod.grid_points(lattice, grid)
    ng = r.shape[0]
    centers = cell.atoms_frac @ lattice
    nao = int(sum((l + 1) * (l + 2) // 2 for l in basis.shell_l))
    chi = np.zeros((kf.shape[0], nao, ng), dtype=np.complex128)
    mu0 = 0
    for s in range(len(basis.shell_l)):
        l = int(basis.shell_l[s])
        alpha = float(basis.shell_exp[s])
        R = centers[int(basis.shell_atom[s])]
        t = shell_images(lattice, R, alpha, l, tol)
        T = t @ lattice
        phase = np.exp(2j * np.pi * (kf @ t.T))                  # exp(i k.T), (nk, nT)
        powers = cartesian_powers(l)
        norms = [component_norm(alpha, *p) for p in powers]
        for n0 in range(0, ng, chunk):
            x = r[None, n0:n0 + chunk, :] - R[None, None, :] - T[:, None, :]   # (nT, nc, 3)
            radial = np.exp(-alpha * np.sum(x * x, axis=2))
            for ic, (a, b, c) in enumerate(powers):
                phi = norms[ic] * x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** c * radial
                chi[:, mu0 + ic, n0:n0 + chunk] = phase @ phi
        mu0 += len(powers)
    return chi


def ao_labels(basis):
    """(shell, component) for every AO, in AO order."""
    out = []
    for s, l in enumerate(basis.shell_l):
        for ic in range(len(cartesian_powers(int(l)))):
            out.append((s, ic))
    return out


def occupied_orbitals_streamed(cell, basis, kmesh, grid, C, tol=1e-12, chunk=1024, points=None):
    """psi[k, i, n] = sum_mu C[k, mu, i] chi[k, mu, n] (paper eq. occmo) without
    holding chi for every k: chi is formed for a slab of grid points at a time
    (the same Bloch sums as ``collocate``) and contracted with C at once.
    ``points`` = (n0, n1) restricts the work to the grid points n0 <= n < n1 (psi
    stays zero elsewhere); it is used only to time a bounded sample."""
    lattice = cell.lattice
    kf = lat_mod.kpoints_fractional(kmesh)
    r = lat_mod.grid_points(lattice, grid)
    ng = r.shape[0]
    centers = cell.atoms_frac @ lattice
    nk, nao, nocc = C.shape
    psi = np.zeros((nk, nocc, ng), dtype=np.complex128)
    shells = []
    for s in range(len(basis.shell_l)):
        l = int(basis.shell_l[s])
        alpha = float(basis.shell_exp[s])
        R = centers[int(basis.shell_atom[s])]
        t = shell_images(lattice, R, alpha, l, tol)
        powers = cartesian_powers(l)
        shells.append((l, alpha, R, t @ lattice, np.exp(2j * np.pi * (kf @ t.T)), powers,
                       [component_norm(alpha, *p) for p in powers]))
    p0, p1 = (0, ng) if points is None else (int(points[0]), min(ng, int(points[1])))
    for n0 in range(p0, p1, chunk):
        rc = r[n0:min(n0 + chunk, p1)]
        chi = np.empty((nk, nao, rc.shape[0]), dtype=np.complex128)
        mu0 = 0
        for (l, alpha, R, T, phase, powers, norms) in shells:
            x = rc[None, :, :] - R[None, None, :] - T[:, None, :]
            radial = np.exp(-alpha * np.sum(x * x, axis=2))
            for ic, (a, b, c) in enumerate(powers):
                phi = norms[ic] * x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** c * radial
                chi[:, mu0 + ic, :] = phase @ phi
            mu0 += len(powers)
        psi[:, :, n0:n0 + rc.shape[0]] = np.matmul(C.transpose(0, 2, 1), chi)
    return psi
