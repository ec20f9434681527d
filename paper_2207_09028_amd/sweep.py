"""Timing sweeps of the three exchange algorithms on one device.

The paper's timing benchmark (Sec. III) times one exchange-matrix build of
diamond with AO-RI-K (Alg. 1), MO-RI-K (Alg. 2) and occ-RI-K (Alg. 3) as the
k-mesh grows, and occ-RI-K alone as the basis grows at a 6x6x6 mesh.  These
sweeps repeat both on the device, all three algorithms through the same pair
passes, kernel multiply and contraction:

  python -m paper_2207_09028_amd.sweep kmesh [--precision fp32split] [--grid 24] [--cap 30]
  python -m paper_2207_09028_amd.sweep basis [--precision fp32split] [--cap 30]
  python -m paper_2207_09028_amd.sweep batch [--precision fp32] [--cells 64] [--small] [--autotune]

The batch sweep times a ragged batch of independent cells (the parallel loop of
Alg. 3 taken over cells): the 64 seeded cells of ``workloads.batch_problems``
(fcc/bcc/rocksalt, 1-4 atoms, 50-350 AOs, 4-8 occupied orbitals, 2^3-4^3 k-meshes,
24^3-48^3 grids), or with ``--small`` the same cells cut to a 2^3 mesh and a 24^3
grid, where launch overheads weigh most.  It reports the builds one after another
on one stream, the same builds spread over the library's worker streams
(occrik_build_batch) and the batch replayed as one HIP graph (occrik_batch_launch).

Inputs are synthetic: the 2-atom diamond cell with even-tempered uncontracted
bases and seeded S-orthonormal occupied coefficients.  Each output line is one
JSON record (algorithm, sizes, pair round trips, ms per build).  A run whose
time, predicted from the algorithm's last measured rate per pair round trip,
exceeds ``--cap`` seconds is reported as skipped.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

import workloads as W

from . import NYQUIST_SYMMETRIC, PREC_FP32, PREC_FP32_SPLIT, PREC_FP64
from .plan import BatchGraph, Plan, PlanSpec, build_batch

PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "fp32split": PREC_FP32_SPLIT}

# per-atom shell counts (s, p, d, f) of the basis sweep and their AO counts for 2 atoms
BASIS_LADDER = [(4, 3), (5, 3, 1), (8, 8, 3), (10, 10, 5, 3), (20, 15, 10, 5)]


def round_trips(algo: str, nk: int, nao: int, nocc: int) -> int:
    """Pair round trips of one build (occ-RI-K with conjugate-pair reuse)."""
    if algo == "occ":
        return nk * nocc * (nk * nocc + 1) // 2
    if algo == "mo":
        return nk * nk * nocc * nao
    return nk * nk * nao * nao


def time_build(plan: Plan, Ct: torch.Tensor, algo: str, reps: int) -> tuple[float, float]:
    """(ms per build, E_x) over ``reps`` builds after one warm-up, timed with events."""
    dev = Ct.device
    K = torch.empty((plan.nk, plan.nao, plan.nao), dtype=torch.complex128, device=dev)
    Ex = torch.empty((1,), dtype=torch.float64, device=dev)
    Kmi = torch.empty((plan.nk, plan.nao, plan.ncol), dtype=torch.complex128, device=dev)

    def once():
        if algo == "occ":
            plan.build_device(Ct, K, Kmi, Ex)
        else:
            plan.conventional_k(Ct, algo=algo, K=K, Ex=Ex)

    once()
    torch.cuda.synchronize()
    if algo == "occ":
        plan.status()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        once()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps, float(Ex[0])


def run_point(prob: W.Problem, algos, precision: int, reps: int, cap: float, rates: dict, tag: dict):
    C = W.random_coefficients(prob)
    Ct = torch.from_numpy(C).to("cuda")
    t0 = time.perf_counter()
    plan = Plan(PlanSpec.from_problem(prob, precision=precision, nyquist=NYQUIST_SYMMETRIC))
    plan_s = time.perf_counter() - t0
    for algo in algos:
        rt = round_trips(algo, prob.nk, prob.nao, prob.nocc)
        rec = dict(tag, algo=algo, nk=prob.nk, nao=prob.nao, nocc=prob.nocc, grid=list(prob.grid),
                   round_trips=rt, plan_s=round(plan_s, 3))
        if algo in rates and rates[algo] * rt * (reps + 1) > cap * 1e3:
            rec["skipped"] = f"predicted {rates[algo] * rt / 1e3:.1f} s per build"
        else:
            ms, ex = time_build(plan, Ct, algo, reps)
            rates[algo] = ms / rt
            rec.update(ms_per_build=round(ms, 3), Ex=ex)
        print(json.dumps(rec), flush=True)
    plan.close()
    del Ct
    torch.cuda.empty_cache()


def sweep_kmesh(args):
    rates: dict = {}
    for m in range(1, args.max_mesh + 1):
        prob = W.Problem(f"kmesh{m}", W.diamond_cell(), W.even_tempered_basis(2, list(args.counts), 0.15, 12.0),
                         (m, m, m), (args.grid,) * 3, args.nocc, seed=100 + m)
        run_point(prob, ("occ", "mo", "ao"), PRECISIONS[args.precision], args.reps, args.cap, rates,
                  dict(sweep="kmesh", precision=args.precision))


def sweep_basis(args):
    rates_big: dict = {}
    rates_small: dict = {}
    for counts in BASIS_LADDER:
        basis = W.even_tempered_basis(2, list(counts), 0.05, 50.0)
        big = W.Problem("basis", W.diamond_cell(), basis, (6, 6, 6), (48, 48, 48), 8, seed=200)
        run_point(big, ("occ",), PRECISIONS[args.precision], args.reps, args.cap, rates_big,
                  dict(sweep="basis", precision=args.precision, counts=list(counts)))
        small = W.Problem("basis", W.diamond_cell(), basis, (2, 2, 2), (48, 48, 48), 8, seed=201)
        run_point(small, ("occ", "mo", "ao"), PRECISIONS[args.precision], args.reps, args.cap, rates_small,
                  dict(sweep="basis", precision=args.precision, counts=list(counts)))


def batch_problems(cells: int, small: bool):
    probs = W.batch_problems(cells)
    if small:
        from dataclasses import replace
        probs = [replace(p, kmesh=(2, 2, 2), grid=(24, 24, 24)) for p in probs]
    return probs


def time_batch(probs, precision: int, reps: int = 3, autotune: bool = False) -> dict:
    """Plans for every cell (Bloch AOs stored), then ms per batch: one build after
    another on one stream, the concurrent batch, the recorded graph's replay and the
    replay of the graph recorded with fused pair-pass rounds (HIP events, each after one
    untimed pass).  Returns a dict of the timings."""
    side = torch.cuda.Stream()
    out = dict(cells=len(probs), precision=int(precision), autotune=bool(autotune))
    with torch.cuda.stream(side):
        t0 = time.perf_counter()
        plans, Cs, Ks, Kmis, Es = [], [], [], [], []
        for p in probs:
            plan = Plan(PlanSpec.from_problem(p, precision=precision, nyquist=NYQUIST_SYMMETRIC))
            Ct = torch.from_numpy(W.random_coefficients(p)).to("cuda")
            plans.append(plan)
            Cs.append(Ct)
            Ks.append(torch.empty((plan.nk, plan.nao, plan.nao), dtype=torch.complex128, device="cuda"))
            Kmis.append(torch.empty((plan.nk, plan.nao, plan.ncol), dtype=torch.complex128, device="cuda"))
            Es.append(torch.empty(1, dtype=torch.float64, device="cuda"))
        side.synchronize()
        out["plan_s"] = round(time.perf_counter() - t0, 3)
        if autotune:
            t0 = time.perf_counter()
            for plan, Ct in zip(plans, Cs):
                plan.autotune(Ct)
            out["autotune_s"] = round(time.perf_counter() - t0, 3)

        def timed(fn):
            fn()
            side.synchronize()
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record(side)
            for _ in range(reps):
                fn()
            stop.record(side)
            side.synchronize()
            return start.elapsed_time(stop) / reps

        def serial():
            for plan, C, K, Kmi, E in zip(plans, Cs, Ks, Kmis, Es):
                plan.build_device(C, K, Kmi, E)

        out["ms_serial"] = round(timed(serial), 3)
        out["ms_concurrent"] = round(timed(lambda: build_batch(plans, Cs, Ks=Ks, Kmis=Kmis, Exs=Es)), 3)
        graph = BatchGraph(plans, Cs, Ks=Ks, Kmis=Kmis, Exs=Es)
        out["ms_graph"] = round(timed(graph.launch), 3)
        for plan in plans:
            plan.status()
        graph.close()
        fused = BatchGraph(plans, Cs, Ks=Ks, Kmis=Kmis, Exs=Es, fused=True)
        out["ms_graph_fused"] = round(timed(fused.launch), 3)
        out["fused_plans"] = fused.fused
        for plan in plans:
            plan.status()
        fused.close()
        out["builds_per_s_graph"] = round(len(probs) / (out["ms_graph"] * 1e-3), 3)
        out["Ex_sum"] = float(sum(float(E[0]) for E in Es))
        for plan in plans:
            plan.close()
    del plans, Cs, Ks, Kmis, Es
    torch.cuda.empty_cache()
    return out


def sweep_batch(args):
    probs = batch_problems(args.cells, args.small)
    rec = dict(sweep="batch", small=bool(args.small), precision=args.precision)
    rec.update(time_batch(probs, PRECISIONS[args.precision], args.reps, args.autotune))
    print(json.dumps(rec), flush=True)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("which", choices=("kmesh", "basis", "batch"))
    ap.add_argument("--precision", choices=tuple(PRECISIONS), default=None,
                    help="fp64, fp32 or fp32split (default fp32split; fp32 for the batch sweep)")
    ap.add_argument("--grid", type=int, default=24, help="grid points per direction (kmesh sweep)")
    ap.add_argument("--counts", type=int, nargs="+", default=[4, 3],
                    help="shells per angular momentum per atom (kmesh sweep)")
    ap.add_argument("--nocc", type=int, default=4, help="occupied orbitals (kmesh sweep)")
    ap.add_argument("--max-mesh", type=int, default=6, help="largest M of the M x M x M meshes")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--cap", type=float, default=30.0, help="seconds; longer runs are skipped")
    ap.add_argument("--cells", type=int, default=64, help="cells of the batch sweep")
    ap.add_argument("--small", action="store_true", help="batch sweep: cut every cell to 2^3 k and 24^3")
    ap.add_argument("--autotune", action="store_true", help="batch sweep: autotune every plan first")
    args = ap.parse_args(argv)
    if args.precision is None:
        args.precision = "fp32" if args.which == "batch" else "fp32split"
    if not torch.cuda.is_available():
        print("the sweeps need a GPU", file=sys.stderr)
        return 2
    np.set_printoptions(precision=4)
    {"kmesh": sweep_kmesh, "basis": sweep_basis, "batch": sweep_batch}[args.which](args)
    return 0


if __name__ == "__main__":
    sys.exit(main())
