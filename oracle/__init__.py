"""FP64 CPU oracle for the occ-RI-K exchange build (TEST INFRASTRUCTURE ONLY).

This package is the plain, slow, obviously-correct reference that the GPU
library is checked against.  It is test infrastructure: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product library never calls it and shares no code with it; the
two meet only in the seeded inputs of the ``workloads`` package.

Modules (each function cites the paper passage it writes out):

* ``lattice``      reciprocal vectors, the real-space grid, G vectors, k-points.
* ``kernels``      reciprocal-space Coulomb kernels f(x) (paper eq. recipcoul) and
                   their omega derivatives.
* ``collocation``  Bloch sums of cartesian Gaussians on the grid (Sec. II.A, first
                   equation; the 1/sqrt(N_k) is dropped, orbitals are per-cell normalised).
* ``occrik``       the occ-RI-K build (Alg. 3): occupied orbitals (eq. occmo), pair
                   potentials (eqs. aodf, Vrao, VGao), W accumulation (eq. occrikinterm),
                   the AO-occ contraction, the occupied block K_ij, the exchange energy,
                   the assembled exchange matrix, Parseval energy and gradients.
* ``conventional`` the conventional GPW exchange matrices: MO-RI-K (Alg. 2) and
                   AO-RI-K (Alg. 1), used to pin the occ-RI-K identities.

Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_pins.py``.  The projector-form assembly
``occrik.assemble_projector`` (not on the GPU path) is pinned by its identities
and, in a complete basis, by the conventional AO-RI-K matrix.
"""
