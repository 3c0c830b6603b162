"""The direction sampler's sin/cos(2 pi u) (an exact octant reduction plus Taylor series, in the
HIP device header) built for the host and checked on every 24-bit uniform against the FP64
library: the sampled directions' accuracy rests on it."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_sincos_turns_exhaustive(tmp_path):
    exe = str(tmp_path / "sincos_turns_check")
    src = os.path.join(ROOT, "tests", "host", "sincos_turns_check.cpp")
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2412_04634_amd", "csrc"),
           src, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=300).stdout.split()
    max_s, max_c = float(out[0]), float(out[1])
    # a few ulp of values up to 1 (ulp 6e-8 on [1/2, 1))
    assert max_s <= 1e-7 and max_c <= 1e-7, (max_s, max_c)
