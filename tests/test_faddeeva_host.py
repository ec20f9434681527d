"""Host (CPU) check of the library's Faddeeva function (Weideman's rational
approximation with compile-time coefficients, used by the truncated long-range
kernel) against scipy.special.wofz over the region that kernel evaluates."""
import os
import subprocess

import numpy as np
import pytest
from scipy.special import wofz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc to build the host test")
def test_faddeeva_matches_scipy(tmp_path):
    exe = tmp_path / "test_faddeeva"
    cmd = [HIPCC, "-x", "c++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
           "-I", os.path.join(ROOT, "paper_2207_09028_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "cpp", "test_faddeeva.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    rng = np.random.default_rng(7)
    # z = -x/(2w) + i w R_c: real parts to a few hundred, imaginary parts 0..12
    x = np.concatenate([rng.uniform(-300, 300, 3000), rng.uniform(-6, 6, 3000), [0.0, 1e-8, -2.0]])
    y = np.concatenate([rng.uniform(0.0, 12.0, 3000), rng.uniform(0.0, 3.0, 3000), [0.0, 5.0, 1e-9]])
    inp = "\n".join(f"{a:.17e} {b:.17e}" for a, b in zip(x, y))
    r = subprocess.run([str(exe)], input=inp, capture_output=True, text=True)
    assert r.returncode == 0
    got = np.array([[float(t) for t in line.split()] for line in r.stdout.strip().splitlines()])
    w = got[:, 0] + 1j * got[:, 1]
    ref = wofz(x + 1j * y)
    rel = np.abs(w - ref) / np.abs(ref)
    assert rel.max() < 5e-14, rel.max()
