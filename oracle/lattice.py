"""Lattice, grid and k-point conventions of the GPW scheme (paper Sec. II.A).

Test infrastructure: see the package docstring.
"""
import numpy as np


def volume(lattice):
    """Unit-cell volume Omega = |det A| (rows of A are the lattice vectors)."""
    return abs(float(np.linalg.det(lattice)))


def reciprocal_vectors(lattice):
    """Rows b_d with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(lattice).T


def grid_points(lattice, grid):
    """r_n = sum_d (n_d / N_d) a_d, row-major over (n_1, n_2, n_3); shape (N_g, 3)."""
    n1, n2, n3 = grid
    f = np.stack(np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2, np.arange(n3) / n3,
                             indexing="ij"), -1).reshape(-1, 3)
    return f @ lattice


def fft_indices(n):
    """Integer frequencies of an n-point DFT: 0..n/2-1, -n/2..-1 (the even-n Nyquist bin is -n/2)."""
    return np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)


def miller_grid(grid):
    """Integer triples m for every DFT output position, row-major; shape (N_g, 3)."""
    m = np.stack(np.meshgrid(*[fft_indices(n) for n in grid], indexing="ij"), -1)
    return m.reshape(-1, 3)


def kpoints_fractional(kmesh):
    """Gamma-centred mesh kappa_d / M_d, row-major over (kappa_1, kappa_2, kappa_3)."""
    idx = np.stack(np.meshgrid(*[np.arange(m) for m in kmesh], indexing="ij"), -1).reshape(-1, 3)
    return idx / np.asarray(kmesh, dtype=float)


def kpoints_cartesian(lattice, kmesh):
    return kpoints_fractional(kmesh) @ reciprocal_vectors(lattice)
