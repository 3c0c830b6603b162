"""The device header's own sin/cos (exact argument reduction plus Taylor series) built for the
host and checked against the FP64 library: the direction sampler's sin/cos(2 pi u) on every
24-bit uniform (the sampled directions' accuracy rests on it), and the FP32 encoding's
sin/cos(pi t) on 4M seeded arguments plus exact values at multiples of 1/2."""
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


def _build_and_run(tmp_path, name):
    exe = str(tmp_path / name)
    src = os.path.join(ROOT, "tests", "host", name + ".cpp")
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2412_04634_amd", "csrc"),
           src, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    return subprocess.run([exe], check=True, capture_output=True, text=True, timeout=300).stdout.split()


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_sincospi_small(tmp_path):
    out = _build_and_run(tmp_path, "sincospi_small_check")
    max_s, max_c, inexact = float(out[0]), float(out[1]), int(out[2])
    assert max_s <= 1e-7 and max_c <= 1e-7, (max_s, max_c)
    assert inexact == 0
