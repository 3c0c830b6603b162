"""Serving policy on the CPU with a simulated executor: admission by budget, continuous batching,
per-stream frame order, release of idle streams, and failure handling."""
import pytest

from paper_2412_04634_amd import serve


class SimExecutor:
    """Simulated device: a batch takes a fixed time per frame plus a fixed overhead; the clock
    advances only when the scheduler submits or idles."""

    def __init__(self, per_frame=0.004, overhead=0.001):
        self.t = 0.0
        self.per_frame, self.overhead = per_frame, overhead
        self.busy_until = 0.0
        self.resident = {}
        self.batches = []
        self.order = {}

    def bytes_for(self, spec):
        return spec.points * 40 + 1000

    def admit(self, spec):
        assert spec.sid not in self.resident
        self.resident[spec.sid] = spec

    def release(self, sid):
        del self.resident[sid]

    def evict(self, sid):
        del self.resident[sid]
        self.evicted = getattr(self, "evicted", 0) + 1

    def now(self):
        return self.t

    def idle(self, next_arrival):
        targets = [x for x in (self.busy_until, next_arrival) if x is not None and x > self.t]
        self.t = min(targets) if targets else self.t + 1e-4

    def submit(self, frames):
        for f in frames:
            assert f.sid in self.resident
            assert self.order.get(f.sid, -1) == f.index - 1     # frames of a stream stay in order
            self.order[f.sid] = f.index
        start = max(self.t, self.busy_until)
        self.busy_until = start + self.overhead + self.per_frame * len(frames)
        self.batches.append(len(frames))
        return self.busy_until

    def poll(self, h):
        return h if self.t >= h else None


def test_all_frames_complete_in_order_with_batching():
    specs = serve.make_stream_specs(5, 16)
    arr = serve.poisson_arrivals(5, 240.0, 2.0, 16)
    ex = SimExecutor()
    sch = serve.Scheduler(specs, ex, budget_bytes=10**12)
    done = sch.run(arr)
    assert len(done) == len(arr)
    assert max(ex.batches) > 1                      # frames of several streams share launches
    for f in done:
        assert f.done >= f.arrival
    st = serve.latency_stats(done)
    assert st["p50_ms"] <= st["p99_ms"]


def test_budget_admission_queues_streams():
    specs = [serve.StreamSpec(i, 100, 100, 4, i) for i in range(6)]
    ex = SimExecutor()
    per = ex.bytes_for(specs[0])
    budget = 2 * per                                  # room for two streams at a time
    arr = [(0.001 * k, k % 6) for k in range(60)]
    sch = serve.Scheduler(specs, ex, budget_bytes=budget)
    done = sch.run(arr)
    assert len(done) == 60
    assert sch.peak_used <= budget
    assert len(sch.admit_log) >= 6                    # every stream got in eventually
    assert len(ex.resident) == 0                      # and was released when done


def test_stream_larger_than_budget_is_an_error():
    specs = [serve.StreamSpec(0, 1000, 1000, 4, 0)]
    with pytest.raises(ValueError):
        serve.Scheduler(specs, SimExecutor(), budget_bytes=10).run([(0.0, 0)])


def test_poisson_rate_and_uniform_streams():
    arr = serve.poisson_arrivals(1, 240.0, 20.0, 16)
    assert abs(len(arr) / 20.0 - 240.0) < 5 * (240.0 / 20.0) ** 0.5
    counts = [0] * 16
    for _, s in arr:
        counts[s] += 1
    assert min(counts) > 0.6 * len(arr) / 16


def test_tight_budget_evicts_idle_streams_and_bounds_latency():
    # a budget of a third of all streams: idle streams are evicted for waiting ones, so no stream
    # waits for another's last frame; every frame completes, in order, within the budget
    specs = serve.make_stream_specs(5, 16)
    arr = serve.poisson_arrivals(6, 240.0, 3.0, 16)
    ex = SimExecutor(per_frame=0.002)
    total = sum(ex.bytes_for(s) for s in specs)
    sch = serve.Scheduler(specs, ex, budget_bytes=total // 3)
    done = sch.run(arr)
    assert len(done) == len(arr)
    assert sch.peak_used <= total // 3
    assert sch.evictions > 0 and ex.evicted == sch.evictions
    lat = serve.latency_stats(done)
    assert lat["p99_ms"] < 200.0, lat
