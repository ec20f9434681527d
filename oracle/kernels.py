"""Reciprocal-space Coulomb kernels (paper Sec. II.A, eq. recipcoul and the G+q=0 rule).

Test infrastructure: see the package docstring.

f(x) for x = |G + q|:
  Coulomb 1/r            : 4 pi / x^2
  short range erfc(wr)/r : 4 pi / x^2 (1 - exp(-x^2 / 4w^2)),  value pi / w^2 at x = 0
  long range  erf(wr)/r  : 4 pi / x^2 exp(-x^2 / 4w^2)
  truncated Coulomb      : 4 pi / x^2 (1 - cos(x R_c)),         value 2 pi R_c^2 at x = 0
                           (1/r inside a sphere of radius R_c, zero outside; the
                           sphere holds the Born-von Karman supercell's volume,
                           4 pi R_c^3 / 3 = N_k Omega; Sec. II.A, Spencer-Alavi kernel)
At x = 0 the paper inserts a finite-size constant chi; for the Coulomb and the
long-range kernels this build sets it to zero (no Madelung shift), for the
short-range and truncated kernels chi is the x -> 0 limit the paper prescribes.
"""
import numpy as np

COULOMB = 0
ERF_LR = 1
ERFC_SR = 2
TRUNC_COULOMB = 3


def truncation_radius(nk, cell_volume):
    """R_c of the truncated Coulomb kernel: the sphere's volume equals N_k Omega."""
    return (3.0 * nk * cell_volume / (4.0 * np.pi)) ** (1.0 / 3.0)


def kernel_values(x2, kind, omega, rcut=None):
    """f at squared momenta x2 (array), with the x = 0 entries set by the chi rule.

    ``rcut`` is R_c, used by the truncated Coulomb kernel only.
    """
    x2 = np.asarray(x2, dtype=np.float64)
    out = np.zeros_like(x2)
    nz = x2 != 0.0
    if kind == COULOMB:
        out[nz] = 4.0 * np.pi / x2[nz]
    elif kind == ERF_LR:
        out[nz] = 4.0 * np.pi / x2[nz] * np.exp(-x2[nz] / (4.0 * omega * omega))
    elif kind == ERFC_SR:
        out[nz] = 4.0 * np.pi / x2[nz] * (-np.expm1(-x2[nz] / (4.0 * omega * omega)))
        out[~nz] = np.pi / (omega * omega)
    elif kind == TRUNC_COULOMB:
        # 1 - cos(t) written as 2 sin^2(t/2), which keeps full relative precision at small t
        x = np.sqrt(x2[nz])
        out[nz] = 8.0 * np.pi / x2[nz] * np.sin(0.5 * x * rcut) ** 2
        out[~nz] = 2.0 * np.pi * rcut * rcut
    else:
        raise ValueError(kind)
    return out


def kernel_domega(x2, kind, omega):
    """d f / d omega, with the same x = 0 convention (zero where f is zeroed)."""
    x2 = np.asarray(x2, dtype=np.float64)
    out = np.zeros_like(x2)
    nz = x2 != 0.0
    w3 = omega ** 3
    if kind in (COULOMB, TRUNC_COULOMB):
        pass
    elif kind == ERF_LR:
        out[nz] = 2.0 * np.pi / w3 * np.exp(-x2[nz] / (4.0 * omega * omega))
    elif kind == ERFC_SR:
        out[nz] = -2.0 * np.pi / w3 * np.exp(-x2[nz] / (4.0 * omega * omega))
        out[~nz] = -2.0 * np.pi / w3
    else:
        raise ValueError(kind)
    return out
