"""Reciprocal-space Coulomb kernels (paper Sec. II.A, eq. recipcoul and the G+q=0 rule).

Test infrastructure: see the package docstring.

f(x) for x = |G + q|:
  Coulomb 1/r            : 4 pi / x^2
  short range erfc(wr)/r : 4 pi / x^2 (1 - exp(-x^2 / 4w^2)),  value pi / w^2 at x = 0
  long range  erf(wr)/r  : 4 pi / x^2 exp(-x^2 / 4w^2)
At x = 0 the paper inserts a finite-size constant chi; for the Coulomb and the
long-range kernels this build sets it to zero (no Madelung shift), for the
short-range kernel chi = pi / w^2 (the x -> 0 limit the paper prescribes).
"""
import numpy as np

COULOMB = 0
ERF_LR = 1
ERFC_SR = 2


def kernel_values(x2, kind, omega):
    """f at squared momenta x2 (array), with the x = 0 entries set by the chi rule."""
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
    else:
        raise ValueError(kind)
    return out


def kernel_domega(x2, kind, omega):
    """d f / d omega, with the same x = 0 convention (zero where f is zeroed)."""
    x2 = np.asarray(x2, dtype=np.float64)
    out = np.zeros_like(x2)
    nz = x2 != 0.0
    w3 = omega ** 3
    if kind == COULOMB:
        pass
    elif kind == ERF_LR:
        out[nz] = 2.0 * np.pi / w3 * np.exp(-x2[nz] / (4.0 * omega * omega))
    elif kind == ERFC_SR:
        out[nz] = -2.0 * np.pi / w3 * np.exp(-x2[nz] / (4.0 * omega * omega))
        out[~nz] = -2.0 * np.pi / w3
    else:
        raise ValueError(kind)
    return out
