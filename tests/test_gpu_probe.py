"""The microbenchmarks behind the measured peaks of the bench line: argument checks; the MFMA
probe's 16-bit accumulations give exactly the closed-form sums (every operand 1.0, so each MFMA
adds K = 32 to each accumulator element); the atomics probe adds exactly where its address rule
says."""
import numpy as np
import pytest
import torch

from tests.common import host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


def test_probe_rejects_bad_arguments(nirc):
    sink = torch.empty(4 * 256, dtype=torch.float32, device="cuda")
    for prec, iters, fmas in ((1, 31, 0), (1, 0, 0), (1, 32, 16), (3, 32, 0)):
        with pytest.raises(nirc.NircError):
            nirc.nirc_probe_mfma(prec, iters, fmas, sink)


@pytest.mark.parametrize("prec", [1, 2])
def test_probe_16bit_sums(nirc, prec):
    iters, blocks = 64, 4
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    flops = nirc.nirc_probe_mfma(prec, iters, 0, sink)
    assert flops == 8 * iters * 4 * blocks * 16384
    lane = np.arange(blocks * 256) % 64
    # 8 chains x 4 accumulator elements x 32 per MFMA x iters, plus the untouched FMA values
    want = 8 * 4 * 32 * iters + 8 * lane + 28
    np.testing.assert_array_equal(host(sink), want.astype(np.float64))


@pytest.mark.parametrize("prec,fmas", [(0, 0), (0, 64), (1, 32), (2, 64)])
def test_probe_runs_finite(nirc, prec, fmas):
    sink = torch.empty(8 * 256, dtype=torch.float32, device="cuda")
    nirc.nirc_probe_mfma(prec, 32, fmas, sink)
    assert np.all(np.isfinite(host(sink)))


def test_probe_atomics_rejects_bad_arguments(nirc):
    buf = torch.zeros(1024, dtype=torch.int64, device="cuda")
    for lpl, reps, blocks in ((3, 1, 1), (32, 1, 1), (1, 0, 1), (1, 1, 0)):
        with pytest.raises(nirc.NircError):
            nirc.nirc_probe_atomics(lpl, reps, blocks, buf)
    with pytest.raises(nirc.NircError):
        nirc.nirc_probe_atomics(1, 1, 1, torch.zeros(1000, dtype=torch.int64, device="cuda"))


@pytest.mark.parametrize("lpl", [1, 4, 16])
def test_probe_atomics_counts(nirc, lpl):
    n, reps, blocks = 1 << 12, 3, 8
    buf = torch.zeros(n, dtype=torch.int64, device="cuda")
    adds = nirc.nirc_probe_atomics(lpl, reps, blocks, buf)
    T = blocks * 256
    i = np.arange(T * reps, dtype=np.int64)
    e = ((i // lpl) * 16 + i % lpl) & (n - 1)
    want = np.bincount(e, minlength=n)
    got = buf.cpu().numpy()
    assert adds == T * reps
    np.testing.assert_array_equal(got, want)
