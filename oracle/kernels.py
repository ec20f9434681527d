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
  truncated long range   : erf(w r)/r inside the same sphere (eq. lrtrunc), i.e.
                           (4 pi / x) int_0^{R_c} erf(w r) sin(x r) dr.  Eq. lrtrunc
                           writes it with erf of complex arguments whose growth
                           cancels against exp(-x^2/4w^2); with the Faddeeva function
                           w(z) = exp(-z^2) erfc(-iz) the same expression reads
                             4 pi / x^2 [exp(-x^2/4w^2) - erf(w R_c) cos(x R_c)
                                         - exp(-w^2 R_c^2) Re(exp(-i x R_c) w(z))],
                           z = -x/(2w) + i w R_c (upper half plane, |w(z)| <= 1),
                           which has no cancellation.  Value at x = 0:
                           4 pi [(R_c^2/2 - 1/(4w^2)) erf(w R_c) + R_c exp(-w^2 R_c^2)/(2 w sqrt(pi))].
                           (The appendix's asymptotic form is not used: its middle
                           term's sign and exponential are misprinted.)
At x = 0 the paper inserts a finite-size constant chi; for the Coulomb and the
long-range kernels it is zero by default, or (Madelung mode) the Madelung
correction the paper cites without a formula: chi = N_k Omega M_s for Coulomb,
with M_s the Madelung constant of the Born-von Karman supercell (the potential a
unit point charge lacks from its periodic images and neutralising background,
by Ewald summation; xi / L for a simple cubic supercell of side L), and
chi = N_k Omega M_s - pi / w^2 for the long-range kernel (Coulomb minus the
short-range kernel's finite x = 0 value).  For the short-range and truncated
kernels chi is the x -> 0 limit the paper prescribes.
"""
import numpy as np
from scipy import special

COULOMB = 0
ERF_LR = 1
ERFC_SR = 2
TRUNC_COULOMB = 3
TRUNC_ERF_LR = 4


def madelung(lattice):
    """Madelung constant M_s > 0 of the point-charge lattice with rows ``lattice``
    (neutralising background), by Ewald summation:
    M_s = -[sum'_T erfc(eta |T|)/|T| + (4 pi / V) sum'_G exp(-G^2/4eta^2)/G^2
            - 2 eta / sqrt(pi) - pi / (eta^2 V)]."""
    from math import erfc
    lattice = np.asarray(lattice, dtype=float)
    vol = abs(np.linalg.det(lattice))
    eta = np.sqrt(np.pi) / vol ** (1.0 / 3.0)
    recip = 2.0 * np.pi * np.linalg.inv(lattice).T
    rcut, gcut = 7.0 / eta, 14.0 * eta

    def triples(rows, cut):
        """Nonzero integer t with every |t @ rows| <= cut inside the ranges
        (|t_d| <= cut |column d of rows^-1|)."""
        inv = np.linalg.inv(rows)
        n = [int(np.ceil(cut * np.linalg.norm(inv[:, d]))) + 1 for d in range(3)]
        rng = [np.arange(-k, k + 1) for k in n]
        t = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)
        return t[np.any(t != 0, axis=1)]

    tr = triples(lattice, rcut)
    T = np.linalg.norm(tr @ lattice, axis=1)
    real = sum(erfc(eta * x) / x for x in T[T <= rcut])
    tg = triples(recip, gcut)
    G2 = np.sum((tg @ recip) ** 2, axis=1)
    sel = G2 <= gcut * gcut
    rec = 4.0 * np.pi / vol * np.sum(np.exp(-G2[sel] / (4.0 * eta * eta)) / G2[sel])
    return -(real + rec - 2.0 * eta / np.sqrt(np.pi) - np.pi / (eta * eta * vol))


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
    elif kind == TRUNC_ERF_LR:
        x = np.sqrt(x2[nz])
        w, R = omega, rcut
        z = -x / (2.0 * w) + 1j * w * R
        tail = np.real(np.exp(-1j * x * R) * special.wofz(z))
        out[nz] = 4.0 * np.pi / x2[nz] * (np.exp(-x2[nz] / (4.0 * w * w)) - special.erf(w * R) * np.cos(x * R)
                                          - np.exp(-w * w * R * R) * tail)
        out[~nz] = 4.0 * np.pi * ((0.5 * R * R - 0.25 / (w * w)) * special.erf(w * R)
                                  + R * np.exp(-w * w * R * R) / (2.0 * w * np.sqrt(np.pi)))
    else:
        raise ValueError(kind)
    return out


def kernel_domega(x2, kind, omega, rcut=None):
    """d f / d omega, with the same x = 0 convention (zero where f is zeroed).

    Truncated long range: (8 sqrt(pi) / x) g(x), g = int_0^{R_c} r exp(-w^2 r^2) sin(x r) dr
    = -dI/dx for I(x) = int_0^{R_c} exp(-w^2 r^2) cos(x r) dr
    = sqrt(pi)/(2w) [exp(-x^2/4w^2) - exp(-w^2 R_c^2) Re(exp(-i x R_c) w(z))], using
    w'(z) = -2 z w(z) + 2i/sqrt(pi); at x = 0, 8 sqrt(pi) int_0^{R_c} r^2 exp(-w^2 r^2) dr.
    """
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
    elif kind == TRUNC_ERF_LR:
        sp = np.sqrt(np.pi)
        w, R = omega, rcut
        x = np.sqrt(x2[nz])
        z = -x / (2.0 * w) + 1j * w * R
        wz = special.wofz(z)
        dwz = -2.0 * z * wz + 2j / sp
        d = np.exp(-1j * x * R) * (-1j * R * wz - dwz / (2.0 * w))
        dI = sp / (2.0 * w) * (-(x / (2.0 * w * w)) * np.exp(-x2[nz] / (4.0 * w * w))
                               - np.exp(-w * w * R * R) * np.real(d))
        out[nz] = -8.0 * sp / x * dI
        out[~nz] = 8.0 * sp * (sp * special.erf(w * R) / (4.0 * w ** 3) - R * np.exp(-w * w * R * R) / (2.0 * w * w))
    else:
        raise ValueError(kind)
    return out
