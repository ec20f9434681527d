#!/usr/bin/env python3
"""occ-RI-K exchange-build throughput on one MI355X.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload paper]

One step is one full exchange build (orbitals, every (k, k') pair round trip,
contraction, FP64 occupied block / Cholesky / assembly / energy) on inputs
already resident in device memory.  The paper-sized workload is the two-atom
diamond cell with 350 AOs, 8 occupied orbitals, a 6x6x6 k-mesh and a 48^3 grid.
Each precision mode gets its own plan (the Bloch AOs are collocated once per
plan, outside the timed region).  The reported value is the builds/s of the
FP32-split mode, valid only when its |dE_x| <= 1e-6 E_h and max|dK| <= 1e-5
against the FP64 mode of the same build; the FP64 builds/s is reported beside
it.  One JSON line is printed on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "occ-RI-K builds/s at 6³k/350AO, FP32-split vs FP64 @|ΔEx|≤1e-6Eh; %roofline"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_mode(prob, C_dev, precision, nyquist, steps, warmup, profile_level, keep_K=False):
    import torch
    from paper_2207_09028_amd.plan import Plan, PlanSpec
    spec = PlanSpec.from_problem(prob, precision=precision, nyquist=nyquist)
    t0 = time.perf_counter()
    plan = Plan(spec)
    plan_s = time.perf_counter() - t0
    dev = plan.device
    K = torch.empty((plan.nk, plan.nao, plan.nao), dtype=torch.complex128, device=dev)
    Kmi = torch.empty((plan.nk, plan.nao, plan.nocc), dtype=torch.complex128, device=dev)
    Ex = torch.empty((1,), dtype=torch.float64, device=dev)
    for _ in range(warmup):
        plan.build_device(C_dev, K, Kmi, Ex)
    torch.cuda.synchronize()
    plan.status()
    plan.set_profiling(profile_level)
    plan.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        plan.build_device(C_dev, K, Kmi, Ex)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.status()
    prof = plan.profile(reset=True)
    info = plan.query()
    out = dict(seconds=dt, builds_per_s=steps / dt, ms_per_build=1e3 * dt / steps, plan_seconds=plan_s,
               Ex=float(Ex.item()), profile=prof, kbatch=info.kbatch,
               bytes_chi=int(info.bytes_chi), bytes_workspace=int(info.bytes_workspace),
               pass_kernels=pass_kernel_names(info, precision))
    Kkeep = K if keep_K else None
    Kmikeep = Kmi
    plan.close()
    del plan
    return out, Kkeep, Kmikeep


SPECIALISED = (24, 30, 32, 36, 40, 48)


def pass_kernel_names(info, precision):
    """Names (as rocprofv3 prints them) of the kernels that run pair passes 1, 2 and 3."""
    from paper_2207_09028_amd import PREC_FP64
    t = "double" if precision == PREC_FP64 else "float"
    g = tuple(info.grid)
    n = g[0] if g[0] == g[1] == g[2] and g[0] in SPECIALISED else 0
    reg = int(info.reg_fft_passes)
    nout = info.nocc + info.nvir
    jc = 8 if nout <= 8 else 16
    if reg & 1:
        p1 = f"pass1r_kernel<{t}, {n}>"
    else:
        p1 = f"pass1g_kernel<{t}, {n}>" if n else f"pass1_kernel<{t}, 0>"
    if reg & 2:
        p2 = f"pass2r_kernel<{n}>"
    else:
        p2 = f"pass2s_kernel<{t}, {n}>" if n else f"pass2_kernel<{t}, 0>"
    if reg & 4:
        p3 = f"pass3r_kernel<{t}, {n}, 8>"
    elif n and nout <= 8:
        p3 = f"pass3s_kernel<{t}, {n}>"
    elif n and nout <= 16:
        p3 = f"pass3f_kernel<{t}, {n}, {jc}>"
    else:
        p3 = f"pass3_kernel<{t}, 0>"
    return [p1, p2, p3]


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from a committed rocprofv3 --pmc summary under
    profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a copy calibration), or None when no
    summary covers it or the kernel's source or its launch set-up has changed since the
    counters were taken."""
    import glob
    from paper_2207_09028_amd.profiling import read_traffic, sources_sha256
    here = os.path.dirname(os.path.abspath(__file__))
    for path in sorted(glob.glob(os.path.join(here, "profiles", "*pmc*.md"))):
        t = read_traffic(path)
        if t.get("kernel") != kernel or "source" not in t:
            continue
        try:
            sha = sources_sha256(t["source"], here)
        except OSError:
            return None
        if sha != t.get("source_sha256"):
            return None
        return float(t["hbm_bytes_per_launch"])
    return None


def cpu_baseline(prob, nblocks, seed=0):
    """Time the FP64 oracle's Alg. 3 inner loops on a bounded sample of the same workload."""
    import numpy as np
    from oracle import occrik
    geo = occrik.Geometry(prob.cell, prob.kmesh, prob.grid)
    rng = np.random.default_rng(seed)
    psi = np.zeros((geo.nk, prob.nocc, geo.ng), dtype=np.complex128)
    ks = [0] + list(range(1, nblocks))
    for k in set(ks):
        psi[k] = rng.standard_normal((prob.nocc, geo.ng)) + 1j * rng.standard_normal((prob.nocc, geo.ng))
    t0 = time.perf_counter()
    occrik.exchange_w(geo, psi, [0], prob.kernel, prob.omega, "symmetric", k1_subset=ks)
    dt = time.perf_counter() - t0
    per_block = dt / len(ks)
    full = per_block * geo.nk * geo.nk
    return dict(value=1.0 / full, unit="builds/s", cores=1, kind="oracle",
                sample=(f"oracle Alg. 3 inner loops for 1 output k-point x {len(ks)} summed k-points "
                        f"({len(ks) * prob.nocc ** 2} pair round trips at {prob.grid[0]}^3, FP64 numpy FFT, "
                        f"synthetic orbitals) in {dt:.1f} s; builds/s extrapolated by the "
                        f"{geo.nk}x{geo.nk}/{len(ks)} block ratio (collocation and contractions excluded)"),
                seconds_sample=dt)


def copy_bandwidth(gib: float = 2.0, reps: int = 5) -> float:
    """Achievable HBM bandwidth: a plain 2 GiB device-to-device copy (read + write bytes)
    timed with events, the measured denominator beside the spec-sheet peak."""
    import torch
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        y.copy_(x)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="paper")
    ap.add_argument("--modes", default="fp64,fp32,fp32split")
    ap.add_argument("--profile-level", type=int, default=2)
    ap.add_argument("--cpu-blocks", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py measures one GPU only: the exchange build runs on a single MI355X and "
              f"--gpus {a.gpus} is not supported", file=sys.stderr)
        return 2
    import numpy as np
    import torch
    import workloads as W
    from paper_2207_09028_amd import PREC_FP32, PREC_FP32_SPLIT, PREC_FP64, NYQUIST_SYMMETRIC

    prob = W.make_problem(a.workload)
    log(f"[bench] workload {a.workload}: nk={prob.nk} nao={prob.nao} nocc={prob.nocc} grid={prob.grid}")
    t0 = time.perf_counter()
    C = W.random_coefficients(prob)
    log(f"[bench] inputs generated in {time.perf_counter() - t0:.1f} s")
    C_dev = torch.from_numpy(C).to("cuda")
    modes = [m.strip() for m in a.modes.split(",") if m.strip()]
    prec = {"fp64": PREC_FP64, "fp32": PREC_FP32, "fp32split": PREC_FP32_SPLIT}
    results, K_ref, Kmi_ref = {}, None, None
    for m in modes:
        log(f"[bench] mode {m}: plan + {a.warmup} warmup + {a.steps} timed builds")
        r, K, Kmi = run_mode(prob, C_dev, prec[m], NYQUIST_SYMMETRIC, a.steps, a.warmup, a.profile_level,
                             keep_K=True)
        if m == "fp64":
            K_ref, Kmi_ref = K, Kmi
        elif K_ref is not None:
            r["dEx_vs_fp64"] = abs(r["Ex"] - results["fp64"]["Ex"])
            r["max_dK_vs_fp64"] = float((K - K_ref).abs().max().item())
            r["max_dKmi_vs_fp64"] = float((Kmi - Kmi_ref).abs().max().item())
        del K, Kmi
        torch.cuda.empty_cache()
        results[m] = r
        log(f"[bench] mode {m}: {r['builds_per_s']:.4f} builds/s ({r['ms_per_build']:.1f} ms/build), "
            f"plan {r['plan_seconds']:.1f} s, Ex={r['Ex']:.12f}")

    # headline: FP32-split when it meets the accuracy gate, else the FP64 number
    head = "fp32split" if "fp32split" in results else modes[0]
    valid = True
    if head != "fp64" and "fp64" in results:
        valid = results[head]["dEx_vs_fp64"] <= 1e-6 and results[head]["max_dK_vs_fp64"] <= 1e-5
    if not valid:
        head = "fp64"
    hr = results[head]
    prof = hr["profile"]
    # dominant pair kernel: the pass with the largest accumulated time
    q = max(range(3), key=lambda i: prof["ms_pass"][i])
    nl = max(1, prof["launches_pass"][q])
    avg_ms = prof["ms_pass"][q] / nl
    bytes_per_launch = prof["bytes_pass"][q] / nl
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    kname = hr["pass_kernels"][q]
    copy_gbs = copy_bandwidth()
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kname), "avg_launch_ms": avg_ms, "bytes_per_launch": bytes_per_launch,
                "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}
    log(f"[bench] device copy {copy_gbs:.0f} GB/s; {kname} {achieved:.0f} GB/s")
    cpu = None
    if not a.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle sample of {a.cpu_blocks} blocks")
        cpu = cpu_baseline(prob, a.cpu_blocks)
        log(f"[bench] cpu baseline {cpu['value']:.3e} builds/s ({cpu['seconds_sample']:.1f} s sample)")
    dtype = {"fp64": "f64", "fp32": "f32", "fp32split": "f32"}[head]
    line = {
        "metric": METRIC, "value": hr["builds_per_s"], "unit": "builds/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": hr["ms_per_build"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": (f"{a.workload}: diamond fcc 2-atom cell, {prob.nao} AO, {prob.nocc} occ, "
                                f"{prob.kmesh[0]}x{prob.kmesh[1]}x{prob.kmesh[2]} k, {prob.grid[0]}^3 grid, "
                                f"kernel {prob.kernel}, nyquist symmetric"),
                   "mode": head, "accuracy_gate_met": valid},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes": {m: {k: v for k, v in r.items() if k != "profile"} | {"ms_pass": r["profile"]["ms_pass"],
                                                                        "launches_pass": r["profile"]["launches_pass"]}
                  for m, r in results.items()},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
