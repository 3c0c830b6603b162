"""The serving loop on the GPU: every frame completes, admission respects the budget, and each
stream's result is the same alone and in the mix (bitwise: the batched launch computes every
request exactly as a single launch does, and each stream's training sees the same frames in the
same order)."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import serve as m
    return m


def test_mix_equals_alone(serve):
    # eight streams under a budget of 40 % of what they would hold together: admission waits,
    # the estimate and the training of each mix run as one replayed graph, and every stream ends
    # exactly where it ends alone
    print("serving mix vs alone", flush=True)
    specs = [serve.StreamSpec(0, 160, 90, 4, 11), serve.StreamSpec(1, 320, 180, 8, 12),
             serve.StreamSpec(2, 64, 64, 32, 13), serve.StreamSpec(3, 200, 100, 16, 14),
             serve.StreamSpec(4, 96, 54, 4, 15), serve.StreamSpec(5, 256, 144, 32, 16),
             serve.StreamSpec(6, 128, 72, 8, 17), serve.StreamSpec(7, 180, 120, 4, 18)]
    ex = serve.GpuExecutor(precision=1, train_batch=4096, train_steps=2)
    ex.keep_final = True
    arrivals = serve.poisson_arrivals(3, 600.0, 0.3, len(specs))
    total = sum(ex.bytes_for(s) for s in specs)
    budget = int(0.4 * total)
    sch = serve.Scheduler(specs, ex, budget)
    done = sch.run(arrivals)
    torch.cuda.synchronize()
    assert len(done) == len(arrivals)
    assert sch.peak_used <= budget < total
    assert any(w > 0 for _, w in sch.admit_waits)          # some stream waited for memory
    assert max(sch.batch_sizes) > 1                         # some frames were trained together
    counts = {}
    for _, sid in arrivals:
        counts[sid] = counts.get(sid, 0) + 1
    for sid, n in counts.items():
        w_mix, out_mix = ex.final[sid]
        w_alone, out_alone = serve.run_alone(ex, specs[sid], n)
        assert torch.equal(w_mix, w_alone), sid
        assert torch.equal(out_mix, out_alone), sid


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


def _models(nirc, prec, sizes, seed0):
    from paper_2412_04634_amd import workload as wl
    out = []
    for i, (P, B) in enumerate(sizes):
        pts = nirc.Points.from_workload(wl.make_points(seed0 + i, P))
        lob = wl.make_lobes(seed0 + i)
        w0 = wl.make_weights(seed0 + i, 64)
        cfg = nirc.make_config(precision=prec, loss_scale=(64.0 if prec == 2 else 1.0), loss=(i % 2))
        out.append(dict(pts=pts, lobes=lob, w0=w0, cfg=cfg, B=B, seed=seed0 + 100 + i))
    return out


def _state(m):
    a, v, step = m.get_adam()
    return m.get_weights().clone(), a.clone(), v.clone(), int(step.item())


@pytest.mark.parametrize("prec", [1, 2])
def test_train_frame_batch_equals_each_alone(nirc, prec):
    # one frame's training of four caches of different sizes, batches and losses in one batched
    # sequence against nirc_train_frame of each alone: bit-identical weights, moments and steps
    print(f"train_frame_batch prec={prec}", flush=True)
    specs = _models(nirc, prec, [(3000, 4096), (700, 1000), (5000, 2048), (4096, 333)], 40)
    maxb = 4096
    mix = [nirc.Model(s["w0"], cfg=s["cfg"], max_batch=maxb) for s in specs]
    alone = [nirc.Model(s["w0"], cfg=s["cfg"], max_batch=s["B"]) for s in specs]
    tb = nirc.TrainBatch(maxb)
    for frame in range(2):
        reqs = [dict(model=m, points=s["pts"], lobes=s["lobes"].rotated(frame).packed(), batch=s["B"],
                     seed=s["seed"], frame=frame) for m, s in zip(mix, specs)]
        tb.set(reqs)
        tb.launch(3)
        for m, s in zip(alone, specs):
            nirc.nirc_train_frame(m, s["pts"], s["lobes"].rotated(frame).packed(), s["B"], 3, s["seed"], frame)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(mix, alone)):
            sa, sb = _state(a), _state(b)
            for x, y in zip(sa[:3], sb[:3]):
                assert torch.equal(x, y), (frame, i)
            assert sa[3] == sb[3] == 3 * (frame + 1)
            assert a.read_flags() == 0


def test_train_frame_batch_graph_replays_other_lists(nirc):
    # a captured training sequence replayed after rewriting its work list with other models and
    # frames computes what eager launches compute (checked on every replay, eager work between)
    specs = _models(nirc, 1, [(2000, 1024), (900, 512), (3000, 2000)], 60)
    maxb = 2048
    ga = [nirc.Model(s["w0"], cfg=s["cfg"], max_batch=maxb) for s in specs]
    ea = [nirc.Model(s["w0"], cfg=s["cfg"], max_batch=maxb) for s in specs]
    tb = nirc.TrainBatch(maxb)
    te = nirc.TrainBatch(maxb)
    graph = None
    plan = [[0, 1, 2], [2, 0], [1], [0, 1, 2], [2]]
    for frame, idx in enumerate(plan):
        tb.set([dict(model=ga[i], points=specs[i]["pts"], lobes=specs[i]["lobes"].packed(), batch=specs[i]["B"],
                     seed=specs[i]["seed"], frame=frame) for i in idx])
        if graph is None:
            tb.launch(2)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            # capturing records the launches without running them: frame 0 ran eagerly above
            with torch.cuda.graph(graph, stream=torch.cuda.Stream()):
                tb.launch(2)
        else:
            graph.replay()
        te.set([dict(model=ea[i], points=specs[i]["pts"], lobes=specs[i]["lobes"].packed(), batch=specs[i]["B"],
                     seed=specs[i]["seed"], frame=frame) for i in idx])
        te.launch(2)
        torch.cuda.synchronize()
        for i in idx:
            assert torch.equal(ga[i].get_weights(), ea[i].get_weights()), (frame, i)
