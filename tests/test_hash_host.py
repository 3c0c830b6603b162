"""Host builds of the hash-grid model's device code (no GPU): the spherical harmonics against the
oracle, and the packed 16-bit weight layout's coverage of the canonical parameters."""
import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _build(tmp_path, name):
    exe = str(tmp_path / name)
    src = os.path.join(ROOT, "tests", "host", name + ".cpp")
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2412_04634_amd", "csrc"),
           src, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    return exe


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_device_sh_matches_oracle(tmp_path):
    exe = _build(tmp_path, "sh25_check")
    rng = np.random.default_rng(3)
    d = rng.normal(size=(5000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d = np.concatenate([d, np.eye(3), -np.eye(3)]).astype(np.float32)
    inp = "\n".join("%.9e %.9e %.9e" % tuple(r) for r in d) + "\n"
    out = subprocess.run([exe], input=inp, check=True, capture_output=True, text=True, timeout=300).stdout
    Y = np.array([[float(v) for v in l.split()] for l in out.strip().split("\n")])
    ref = oracle.sh(d.astype(np.float64))
    # FP32 polynomials on FP32 unit vectors: a few ulp of values below 1
    assert np.abs(Y - ref).max() <= 2e-6


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_hash_packed_layout_covers_parameters(tmp_path):
    exe = _build(tmp_path, "hash_layout_check")
    lines = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=300).stdout.split("\n")
    total, secD, rest, secTS, secT0 = (int(v) for v in lines[0].split())
    src = np.array([int(v) for v in lines[1:total + 1]])
    W, nin = 64, 64
    w1 = W * nin
    # W1 surface + direction sections: every W1 entry exactly once (inputs 0..63)
    s1 = src[:rest]
    s1 = s1[s1 >= 0]
    assert sorted(s1.tolist()) == list(range(w1))
    # direction section holds the SH columns 24..48, surface section the others
    d = src[secD:rest]
    d = d[d >= 0]
    assert set((d % nin).tolist()) == set(range(24, 49))
    # hidden layers: W2..W4 twice (forward H and transposed T), W5 in O, OS (x4 copies) and OT
    h = src[rest:secTS]
    h = h[h >= 0]
    counts = np.bincount(h, minlength=w1 + 3 * W * W + 3 * W)
    assert (counts[:w1] == 0).all()
    assert (counts[w1:w1 + 3 * W * W] == 2).all()
    assert (counts[w1 + 3 * W * W:] >= 3).all()
    # TS: the grid columns of W1 (inputs 0..23), each once
    ts = src[secTS:]
    ts = ts[ts >= 0]
    assert sorted(ts.tolist()) == sorted(r * nin + c for r in range(W) for c in range(24))
    assert secT0 > rest
    # FP32 layout: surface + direction sections hold W1 once, the hidden sections W2..W4 twice
    # (forward and transposed) and W5 in O and OT, the TS32 section W1's grid columns once
    total32, rest32, ts32 = (int(v) for v in lines[total + 1].split())
    src32 = np.array([int(v) for v in lines[total + 2:total + 2 + total32]])
    s1 = src32[:rest32]
    assert sorted(s1[s1 >= 0].tolist()) == list(range(w1))
    h = src32[rest32:ts32]
    counts = np.bincount(h[h >= 0], minlength=w1 + 3 * W * W + 3 * W)
    assert (counts[:w1] == 0).all()
    assert (counts[w1:w1 + 3 * W * W] == 2).all()
    assert (counts[w1 + 3 * W * W:] >= 2).all()
    ts = src32[ts32:]
    assert sorted(ts[ts >= 0].tolist()) == sorted(r * nin + c for r in range(W) for c in range(24))


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("grid", [(18, 16, 1.5), (10, 4, 1.5)])
def test_device_grid_lookup_matches_oracle(tmp_path, grid):
    # the kernels' grid fetch and trilinear blend (FP32) against the oracle's encoding (FP64), on
    # random features in [-1, 1] and positions inside and outside the unit cube
    from paper_2412_04634_amd import workload as wl
    exe = _build(tmp_path, "hash_grid_check")
    n = oracle.hash_entries(grid)
    rng = np.random.default_rng(11)
    table = rng.uniform(-1.0, 1.0, 2 * n).astype(np.float32)
    pts = wl.make_points(12, 3000)
    xyz = np.stack([pts.px, pts.py, pts.pz], axis=1).astype(np.float32)
    xyz[:200] = (xyz[:200] * 1.4 - 0.2).astype(np.float32)
    pts.px[:], pts.py[:], pts.pz[:] = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    ft, fp = str(tmp_path / "table.bin"), str(tmp_path / "pts.bin")
    table.tofile(ft)
    np.ascontiguousarray(xyz).tofile(fp)
    run = subprocess.run([exe, ft, fp, str(grid[0]), str(grid[1]), str(grid[2])], check=True, capture_output=True,
                         text=True, timeout=300)
    out = run.stdout
    # the training scatter's corner entries and weights agree with the fetch corner by corner
    mismatch, max_w = run.stderr.split()
    assert int(mismatch) == 0 and float(max_w) <= 1e-5
    got = np.array([[float(v) for v in l.split()] for l in out.strip().split("\n")])
    ref = oracle.hash_encode(pts, None, np.tile([[0.0, 0.0, 1.0]], (3000, 1)), table.astype(np.float64), grid)[:, :24]
    # level l: the FP32 product x N_l is off by up to half an ulp (2^-24 N_l relative to the cell),
    # which moves the blend of features in [-1, 1] by at most that times the largest corner
    # difference (2) along each axis; the blend itself adds a few 1e-7
    res, _, _ = oracle.hash_levels(grid)
    err = np.abs(got - ref)
    for l in range(12):
        bound = 3 * 2 * 2.0 ** -24 * float(res[l]) * 2 + 1e-6
        assert err[:, 2 * l:2 * l + 2].max() <= bound, (l, err[:, 2 * l:2 * l + 2].max(), bound)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_h16_packed_targets_invert_the_packing(tmp_path):
    # the per-parameter lists of packed elements (used to refresh the kernels' copies right after
    # each Adam update) are exactly the inverses of the packings, 16-bit scales included, at both
    # widths and in both layouts
    exe = _build(tmp_path, "h16_targets_check")
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=300).stdout.split("\n")
    rows = [list(map(int, l.split())) for l in out if l.strip()]
    h16 = [r for r in rows if len(r) == 5]
    f32 = [r[1:] for r in rows if len(r) == 6 and r[0] == 32]
    assert [r[0] for r in h16] == [64, 128] and [r[0] for r in f32] == [64, 128]
    for W, bad, np_, used, listed in h16 + f32:
        assert bad == 0, (W, bad)
        assert used == listed   # every stored element is some parameter's target
        assert np_ == W * 160 + 3 * W * W + 3 * W
    for W, bad, np_, used, listed in f32:
        assert listed == np_ + 3 * W * W + 3 * W   # W2..W5 twice (forward and transposed)
