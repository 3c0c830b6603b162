"""Continuous batching: one persistent launch over several streams' frames (needs the GPU).

Each request in a mixed batch must produce exactly (bitwise) what tlmc_estimate gives for it
alone; a captured launch replayed after rewriting the work list must do the same.
"""
import numpy as np
import pytest
import torch

from paper_2412_04634_amd import workload as wl

pytestmark = pytest.mark.gpu
W = 64


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


def make_streams(nirc, prec, specs):
    out = []
    for i, (P, N) in enumerate(specs):
        pts = nirc.Points.from_workload(wl.make_points(100 + i, P))
        lob = wl.make_lobes(100 + i).rotated(3 * i).packed()
        model = nirc.Model(wl.make_weights(200 + i, W), cfg=nirc.make_config(precision=prec), max_batch=0)
        out.append(dict(model=model, points=pts, lobes=lob, n_cache=N, seed=7 + i, frame=i,
                        out_tl=torch.full((P, 3), -1.0, device="cuda"),
                        out_c=torch.full((P, 3), -1.0, device="cuda"),
                        out_r=torch.full((P, 3), -1.0, device="cuda")))
    return out


SPECS = [(640 * 36, 4), (1000, 8), (17, 32), (4096, 16), (1, 1), (5000, 3), (2048, 64)]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batch_equals_alone(nirc, prec):
    print(f"batch prec={prec}", flush=True)
    reqs = make_streams(nirc, prec, SPECS)
    b = nirc.Batch()
    b.set(reqs)
    b.launch()
    for r in reqs:
        tl, c, rr = nirc.tlmc_estimate(r["model"], r["points"], r["lobes"], r["n_cache"], r["seed"], r["frame"],
                                       parts=True)
        assert torch.equal(r["out_tl"], tl)
        assert torch.equal(r["out_c"], c)
        assert torch.equal(r["out_r"], rr)


def test_batch_graph_replay_with_changing_mix(nirc):
    print("batch graph replay", flush=True)
    reqs = make_streams(nirc, 1, SPECS)
    b = nirc.Batch()
    b.set(reqs[:3])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.launch()          # warm-up on the capture stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.launch()
    mixes = [reqs[:3], reqs[3:], [reqs[1], reqs[5]], reqs]
    for it, mix in enumerate(mixes):
        for r in mix:
            r["out_tl"].fill_(-1.0)
        for r in mix:
            r["frame"] += 1
        b.set(mix)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for r in mix:
            tl = nirc.tlmc_estimate(r["model"], r["points"], r["lobes"], r["n_cache"], r["seed"], r["frame"])
            assert torch.equal(r["out_tl"], tl), (it, r["n_cache"])


def test_batch_rejects_mixed_precision(nirc):
    a = make_streams(nirc, 0, SPECS[:1])
    c = make_streams(nirc, 1, SPECS[1:2])
    with pytest.raises(nirc.NircError):
        nirc.Batch().set(a + c)
