"""Profiling helpers run under rocprofv3.

    python -m paper_2207_09028_amd.profiling copy [--gib 2]
        a plain device-to-device copy of a known size, whose FETCH_SIZE /
        WRITE_SIZE counters calibrate the HBM-traffic counters of the library
        kernels (bytes counted per byte actually moved);
    python -m paper_2207_09028_amd.profiling summarize <kernel_stats.csv> [--top 12]
        a short text table of a rocprofv3 --stats kernel summary;
    python -m paper_2207_09028_amd.profiling traffic --kernel NAME --source FILE[,FILE...] \
            <fetch.csv> <write.csv> <copy_fetch.csv> <copy_write.csv>
        HBM bytes per dispatch of one kernel from two rocprofv3 --pmc runs
        (FETCH_SIZE, WRITE_SIZE), each scaled by what the same counter reads for
        the plain copy above; prints "key: value" lines that bench.py reads back
        (with one SHA-256 over the kernel's source and the files that set its
        launch, in the order given, so a changed kernel or launch reads as
        unmeasured);
    python -m paper_2207_09028_amd.profiling phases <fetch.csv> <write.csv> \
            <copy_fetch.csv> <copy_write.csv> <kernel_stats.csv>
        the same measured bytes for every pair pass and contraction kernel, with
        the achieved GB/s over the kernel trace's average duration.
"""
from __future__ import annotations

import argparse
import csv
import sys


def copy(gib: float, reps: int = 3):
    import torch
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {reps} x {n * 4} bytes")


def summarize(path: str, top: int = 12):
    rows = list(csv.DictReader(open(path)))
    key_t = next(k for k in rows[0] if k.lower().startswith("totaldurationns"))
    key_n = next(k for k in rows[0] if k.lower() == "calls")
    key_a = next(k for k in rows[0] if k.lower().startswith("averagens"))
    rows.sort(key=lambda r: -float(r[key_t]))
    total = sum(float(r[key_t]) for r in rows)
    print(f"{'kernel':60s} {'calls':>7s} {'avg_ms':>10s} {'total_ms':>10s} {'share':>6s}")
    for r in rows[:top]:
        name = r["Name"][:60]
        print(f"{name:60s} {int(r[key_n]):7d} {float(r[key_a]) / 1e6:10.3f} {float(r[key_t]) / 1e6:10.1f} "
              f"{100 * float(r[key_t]) / total:5.1f}%")


def _counter_per_dispatch(path: str, counter: str, kernel: str):
    """(mean counter value per dispatch, dispatches) over rows whose kernel name contains ``kernel``."""
    tot, n = 0.0, 0
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter and kernel in r["Kernel_Name"]:
            tot += float(r["Counter_Value"])
            n += 1
    return (tot / n if n else 0.0), n


def _copy_scale(path: str, counter: str, nbytes: int):
    """Bytes actually moved per counter unit (KiB) for the calibration copy."""
    val, n = _counter_per_dispatch(path, counter, "copyBuffer")
    if n == 0:
        val, n = _counter_per_dispatch(path, counter, "copy")
    return nbytes / (val * 1024.0) if val else float("nan")


def sources_sha256(sources: str, root: str = "") -> str:
    """SHA-256 over the bytes of the comma-separated files ``sources``, concatenated in order."""
    import hashlib
    import os
    h = hashlib.sha256()
    for f in sources.split(","):
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic(kernel: str, source: str, fetch_csv: str, write_csv: str, cfetch_csv: str, cwrite_csv: str,
            copy_gib: float = 2.0):
    import hashlib
    nbytes = int(copy_gib * (1 << 30)) // 4 * 4
    fs = _copy_scale(cfetch_csv, "FETCH_SIZE", nbytes)
    ws = _copy_scale(cwrite_csv, "WRITE_SIZE", nbytes)
    f, nf = _counter_per_dispatch(fetch_csv, "FETCH_SIZE", kernel)
    w, nw = _counter_per_dispatch(write_csv, "WRITE_SIZE", kernel)
    sha = sources_sha256(source)
    total = f * 1024.0 * fs + w * 1024.0 * ws
    print(f"kernel: {kernel}")
    print(f"source: {source}")
    print(f"source_sha256: {sha}")
    print(f"dispatches: {nf} {nw}")
    print(f"fetch_size_kib_per_dispatch: {f:.1f}")
    print(f"write_size_kib_per_dispatch: {w:.1f}")
    print(f"fetch_scale: {fs:.4f}")
    print(f"write_scale: {ws:.4f}")
    print(f"hbm_bytes_per_launch: {total:.6e}")


def phases(fetch_csv: str, write_csv: str, cfetch_csv: str, cwrite_csv: str, stats_csv: str,
           kernels=("pass1", "pass2", "pass3", "wreduce", "kvals", "kcache", "orbitals_mfma", "contract_mfma"),
           copy_gib: float = 2.0):
    """Measured HBM bytes per dispatch (counters, copy-calibrated) and achieved GB/s over the
    kernel-trace average duration, for every kernel whose name contains one of ``kernels``."""
    import collections
    import re
    nbytes = int(copy_gib * (1 << 30)) // 4 * 4
    fs = _copy_scale(cfetch_csv, "FETCH_SIZE", nbytes)
    ws = _copy_scale(cwrite_csv, "WRITE_SIZE", nbytes)

    def per_kernel(path, counter):
        acc = collections.defaultdict(lambda: [0.0, 0])
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                m = re.search(r"(\w+<[^()]*>)\(", r["Kernel_Name"])
                k = m.group(1) if m else r["Kernel_Name"].split("(")[0]
                acc[k][0] += float(r["Counter_Value"])
                acc[k][1] += 1
        return acc

    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    rows = list(csv.DictReader(open(stats_csv)))
    key_a = next(k for k in rows[0] if k.lower().startswith("averagens"))
    avg = {}
    for r in rows:
        m = re.search(r"(\w+<[^()]*>)\(", r["Name"])
        avg[m.group(1) if m else r["Name"].split("(")[0]] = float(r[key_a]) / 1e6
    print(f"{'kernel':36s} {'disp':>5s} {'read GB':>9s} {'write GB':>9s} {'avg ms':>8s} {'GB/s':>8s}")
    for k in sorted(fetch, key=lambda k: -(fetch[k][0] / max(fetch[k][1], 1))):
        if not any(s in k for s in kernels) or k not in avg:
            continue
        f = fetch[k][0] / fetch[k][1] * 1024.0 * fs
        w = write[k][0] / max(write[k][1], 1) * 1024.0 * ws
        print(f"{k:36s} {fetch[k][1]:5d} {f / 1e9:9.3f} {w / 1e9:9.3f} {avg[k]:8.3f} {(f + w) / (avg[k] * 1e6):8.1f}")


def read_traffic(path: str) -> dict:
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#", "|", "`")):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--gib", type=float, default=2.0)
    s = sub.add_parser("summarize")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=12)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--source", required=True)
    t.add_argument("--copy-gib", type=float, default=2.0)
    t.add_argument("csvs", nargs=4)
    ph = sub.add_parser("phases")
    ph.add_argument("--copy-gib", type=float, default=2.0)
    ph.add_argument("csvs", nargs=5, help="fetch write copy-fetch copy-write kernel-stats")
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy(a.gib)
    elif a.cmd == "traffic":
        traffic(a.kernel, a.source, *a.csvs, copy_gib=a.copy_gib)
    elif a.cmd == "phases":
        phases(*a.csvs, copy_gib=a.copy_gib)
    else:
        summarize(a.csv, a.top)


if __name__ == "__main__":
    sys.exit(main())
