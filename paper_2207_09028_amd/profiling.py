"""Profiling helpers run under rocprofv3.

    python -m paper_2207_09028_amd.profiling copy [--gib 2]
        a plain device-to-device copy of a known size, whose FETCH_SIZE /
        WRITE_SIZE counters calibrate the HBM-traffic counters of the library
        kernels (bytes counted per byte actually moved);
    python -m paper_2207_09028_amd.profiling bandwidth [--gib 4] [--reps 10]
        the library's streaming probe kernels (occrik_hbm_probe): read-only,
        write-only and copy rates with 8- and 16-byte lane accesses, temporal
        and non-temporal, timed with HIP events; the achievable roofs of the
        write-heavy pass 1, the read-heavy pass 3 and the balanced pass 2;
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
        the achieved GB/s over the kernel trace's average duration;
    python -m paper_2207_09028_amd.profiling counters <counter.csv> [<kernel_stats.csv>] \
            [--kernels pass1,pass2,pass3,orbitals_mfma,contract_mfma]
        the mean per dispatch of every counter of one rocprofv3 --pmc run for the
        kernels named, with the derived rates (VALU instructions per SIMD-cycle,
        LDS bank-conflict cycles per LDS instruction) when the trace's average
        durations are given.
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


def bandwidth(gib: float = 4.0, reps: int = 10):
    """Achievable HBM rates from the library's probe kernels (bytes moved per second:
    reads + writes for the copy)."""
    import ctypes

    import torch

    from . import _lib
    lib = _lib.load()
    nbytes = int(gib * (1 << 30)) // 16 * 16
    a = torch.zeros(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.zeros_like(a)
    torch.cuda.synchronize()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    names = {0: "read", 1: "write", 2: "copy"}
    print(f"{'kind':6s} {'width':>5s} {'nt':>3s} {'GiB':>6s} {'ms':>9s} {'GB/s':>8s}")
    out = {}
    for kind in (0, 1, 2):
        for width in (8, 16):
            for nt in (0, 1):
                ms = ctypes.c_double()
                _lib.check(lib.occrik_hbm_probe(kind, width, nt, 0, ctypes.c_void_p(b.data_ptr()),
                                                ctypes.c_void_p(a.data_ptr()), nbytes, reps, stream,
                                                ctypes.byref(ms)))
                moved = nbytes * (2 if kind == 2 else 1)
                gbs = moved / (ms.value * 1e-3) / 1e9
                out[(names[kind], width, nt)] = gbs
                print(f"{names[kind]:6s} {width:5d} {nt:3d} {gib:6.2f} {ms.value:9.3f} {gbs:8.1f}", flush=True)
    # a write stream with one read for every `every` writes (pass 1 reads about one for eight)
    print(f"\n{'writes per read':>16s} {'nt':>3s} {'write GB/s':>11s} {'read GB/s':>10s} {'total GB/s':>11s}")
    for every in (64, 16, 8, 4, 2, 1):
        for nt in (0, 1):
            ms = ctypes.c_double()
            _lib.check(lib.occrik_hbm_probe(3, 16, nt, every, ctypes.c_void_p(b.data_ptr()),
                                            ctypes.c_void_p(a.data_ptr()), nbytes, reps, stream, ctypes.byref(ms)))
            w = nbytes / (ms.value * 1e-3) / 1e9
            r = w / every
            out[("mixed", every, nt)] = w + r
            print(f"{every:16d} {nt:3d} {w:11.1f} {r:10.1f} {w + r:11.1f}", flush=True)
    return out


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


CLOCK_HZ = 2.4e9       # MI355X peak engine clock
SIMDS = 256 * 4         # 256 CUs, 4 SIMDs each


def _kernel_key(name: str) -> str:
    import re
    m = re.search(r"(\w+<[^()]*>)\(", name)
    return m.group(1) if m else name.split("(")[0]


def counters(counter_csv: str, stats_csv: str | None = None,
             kernels=("pass1", "pass2", "pass3", "orbitals_mfma", "contract_mfma")):
    """Mean value per dispatch of every counter in ``counter_csv`` for the kernels whose
    name contains one of ``kernels``; with the kernel trace's stats, also the VALU issue
    rate per SIMD-cycle (one wave64 VALU instruction every 4 cycles is 0.25) and LDS
    bank-conflict cycles per LDS instruction."""
    import collections
    acc = collections.defaultdict(lambda: collections.defaultdict(lambda: [0.0, 0]))
    for r in csv.DictReader(open(counter_csv)):
        k = _kernel_key(r["Kernel_Name"])
        if not any(s in k for s in kernels):
            continue
        a = acc[k][r["Counter_Name"]]
        a[0] += float(r["Counter_Value"])
        a[1] += 1
    avg = {}
    if stats_csv:
        rows = list(csv.DictReader(open(stats_csv)))
        key_a = next(k for k in rows[0] if k.lower().startswith("averagens"))
        avg = {_kernel_key(r["Name"]): float(r[key_a]) for r in rows}
    for k in sorted(acc):
        print(f"{k}")
        mean = {c: v[0] / max(v[1], 1) for c, v in acc[k].items()}
        for c in sorted(mean):
            print(f"    {c:36s} {mean[c]:16.6g}   ({acc[k][c][1]} dispatches)")
        ns = avg.get(k)
        if ns:
            print(f"    {'trace average duration (ms)':36s} {ns / 1e6:16.4f}")
            if "SQ_INSTS_VALU" in mean:
                ipc = mean["SQ_INSTS_VALU"] / (ns * 1e-9 * CLOCK_HZ * SIMDS)
                print(f"    {'VALU instructions per SIMD-cycle':36s} {ipc:16.4f}   (0.25 = every 4th cycle)")
        if mean.get("SQ_INSTS_LDS"):
            if "SQ_LDS_BANK_CONFLICT" in mean:
                print(f"    {'bank-conflict cycles per LDS instr':36s} "
                      f"{mean['SQ_LDS_BANK_CONFLICT'] / mean['SQ_INSTS_LDS']:16.4f}")


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
    bw = sub.add_parser("bandwidth")
    bw.add_argument("--gib", type=float, default=4.0)
    bw.add_argument("--reps", type=int, default=10)
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
    cn = sub.add_parser("counters")
    cn.add_argument("csvs", nargs="+", help="counter csv [kernel stats csv]")
    cn.add_argument("--kernels", default="pass1,pass2,pass3,orbitals_mfma,contract_mfma")
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy(a.gib)
    elif a.cmd == "traffic":
        traffic(a.kernel, a.source, *a.csvs, copy_gib=a.copy_gib)
    elif a.cmd == "bandwidth":
        bandwidth(a.gib, a.reps)
    elif a.cmd == "phases":
        phases(*a.csvs, copy_gib=a.copy_gib)
    elif a.cmd == "counters":
        counters(a.csvs[0], a.csvs[1] if len(a.csvs) > 1 else None, tuple(a.kernels.split(",")))
    else:
        summarize(a.csv, a.top)


if __name__ == "__main__":
    sys.exit(main())
