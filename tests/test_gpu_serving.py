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
    print("serving mix vs alone", flush=True)
    specs = [serve.StreamSpec(0, 160, 90, 4, 11), serve.StreamSpec(1, 320, 180, 8, 12),
             serve.StreamSpec(2, 64, 64, 32, 13), serve.StreamSpec(3, 200, 100, 16, 14)]
    ex = serve.GpuExecutor(precision=1, train_batch=4096, train_steps=2)
    ex.keep_final = True
    arrivals = serve.poisson_arrivals(3, 400.0, 0.25, len(specs))
    budget = 2 * max(ex.bytes_for(s) for s in specs)      # at most two streams resident at once
    sch = serve.Scheduler(specs, ex, budget)
    done = sch.run(arrivals)
    torch.cuda.synchronize()
    assert len(done) == len(arrivals)
    assert sch.peak_used <= budget
    counts = {}
    for _, sid in arrivals:
        counts[sid] = counts.get(sid, 0) + 1
    for sid, n in counts.items():
        w_mix, out_mix = ex.final[sid]
        w_alone, out_alone = serve.run_alone(ex, specs[sid], n)
        assert torch.equal(w_mix, w_alone), sid
        assert torch.equal(out_mix, out_alone), sid
