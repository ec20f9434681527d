"""Profiling helpers run under rocprofv3.

    python -m paper_2207_09028_amd.profiling copy [--gib 2]
        a plain device-to-device copy of a known size, whose FETCH_SIZE /
        WRITE_SIZE counters calibrate the HBM-traffic counters of the library
        kernels (bytes counted per byte actually moved);
    python -m paper_2207_09028_amd.profiling summarize <kernel_stats.csv> [--top 12]
        a short text table of a rocprofv3 --stats kernel summary.
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--gib", type=float, default=2.0)
    s = sub.add_parser("summarize")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=12)
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy(a.gib)
    else:
        summarize(a.csv, a.top)


if __name__ == "__main__":
    sys.exit(main())
