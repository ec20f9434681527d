"""Write the stored oracle results used by the GPU parity tests at full workload sizes.

    python tests/golden/make_golden.py [prec] [diff] [batch] [paper]

Calls only ``oracle`` (and the seeded ``workloads`` generators); nothing here
comes from the GPU library.  Outputs (numpy .npz, no pickles):

  prec.npz   full build of the 3x3x3 k, 100 AO, 36^3 workload (symmetric Nyquist)
  diff.npz   full build of the 4x4x4 k, 200 AO, 40^3 long-range workload with dE_x/domega
  batch.npz  full builds of the eight capped cells of the ragged batch
             (workloads.batch_parity_problems): per cell i, Kmi_i, Kij_i, Ex_i and
             the rows Krows_i of K~ at the k-points Kk_i
  paper.npz  the 6x6x6 k, 350 AO, 48^3 workload sampled on two output k-points
             (Gamma and k index 43): K_{mu j}(k), K_ij(k), the per-k energy terms
             and every ninth row of the assembled K~(k); every sampled quantity
             sums over all 216 summed k-points, so it is exact, not an estimate.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W                       # noqa: E402
from oracle import collocation, occrik      # noqa: E402

PAPER_K = [0, 43]
PAPER_K_ROWS = np.arange(0, 350, 9)          # rows of K~(k) kept (every ninth AO)


def full(name, domega=False):
    prob = W.make_problem(name)
    C = W.random_coefficients(prob)
    t0 = time.time()
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol)
    res = occrik.build(prob, C, chi=chi, nyquist="symmetric", parseval=True, domega=domega)
    del chi
    out = dict(Kmi=res["Kmi"], Kij=res["Kij"], ex_terms=res["ex_terms"], Ex=res["Ex"],
               Ex_parseval=res["Ex_parseval"], K_sample=res["K"][:2], seconds=time.time() - t0)
    if domega:
        out["dEx_domega"] = res["dEx_domega"]
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), **out)
    print(name, "Ex", res["Ex"], "seconds", out["seconds"], flush=True)


def batch():
    out = {}
    t0 = time.time()
    for i, prob in enumerate(W.batch_parity_problems()):
        C = W.random_coefficients(prob)
        res = occrik.build(prob, C, nyquist="symmetric")
        ks = np.array([0, prob.nk - 1])
        rows = np.arange(0, prob.nao, max(1, prob.nao // 8))
        out.update({f"Kmi_{i}": res["Kmi"], f"Kij_{i}": res["Kij"], f"Ex_{i}": res["Ex"],
                    f"Kk_{i}": ks, f"Krows_{i}": rows, f"K_{i}": res["K"][ks][:, rows]})
        print(prob.name, "Ex", res["Ex"], "seconds", time.time() - t0, flush=True)
    np.savez_compressed(os.path.join(HERE, "batch.npz"), **out)


def paper():
    prob = W.make_problem("paper")
    C = W.random_coefficients(prob)
    t0 = time.time()
    psi = collocation.occupied_orbitals_streamed(prob.cell, prob.basis, prob.kmesh, prob.grid, C,
                                                 prob.lattice_tol)
    t1 = time.time()
    print("paper: orbitals", t1 - t0, flush=True)
    geo = occrik.Geometry(prob.cell, prob.kmesh, prob.grid)
    Wk, _, _ = occrik.exchange_w(geo, psi, PAPER_K, prob.kernel, prob.omega, "symmetric")
    t2 = time.time()
    print("paper: pair loops", t2 - t1, flush=True)
    chi = collocation.collocate(prob.cell, prob.basis, prob.kmesh, prob.grid, prob.lattice_tol,
                                kpoint_indices=PAPER_K)
    Kmi = occrik.contract(geo, chi, Wk)
    Kij = occrik.occupied_block(C[PAPER_K], Kmi)
    terms = occrik.exchange_energy_terms(Kij, geo.nk)
    K = occrik.assemble(Kmi, Kij)
    np.savez_compressed(os.path.join(HERE, "paper.npz"), k=np.array(PAPER_K), Kmi=Kmi, Kij=Kij,
                        ex_terms=terms, K_rows=PAPER_K_ROWS, K=K[:, PAPER_K_ROWS], seconds=time.time() - t0)
    print("paper: done", time.time() - t0, "terms", terms, flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["prec", "diff", "batch", "paper"]
    for w in which:
        if w == "prec":
            full("prec")
        elif w == "diff":
            full("diff", domega=True)
        elif w == "batch":
            batch()
        elif w == "paper":
            paper()
