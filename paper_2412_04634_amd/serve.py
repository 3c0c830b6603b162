"""Multi-stream serving of the two-level estimator: several render streams, each with its own
cache (model + Adam state) resident on the GPU, frames arriving over time.

* Admission by HBM budget: a stream is admitted (its points, outputs, model state and training
  workspace are allocated) only when its resident bytes fit in what the budget has left.  When
  the stream at the head of the waiting queue does not fit, idle resident streams (no frame
  pending or in flight) are evicted, least recently used first: the training state goes to host
  memory (the checkpoint blob) and comes back bit for bit when the stream is admitted again.  A
  stream that has no more frames releases its memory for good.
* Continuous batching: whenever the device can take more work, the oldest pending frame of
  every admitted stream is put into one estimate work list and one training work list; the
  whole frame of the mix - one persistent estimate launch (tlmc_estimate_batch) and each
  training step of all those streams at once (nirc_train_frame_batch) - is one captured graph,
  replayed for every mix after the lists are rewritten.  Frames that arrive meanwhile join the
  next batch.  A stream's frames stay in order (frame f + 1 uses the weights trained after
  frame f).
* Latency of a frame = GPU completion time of its training - its arrival time; reported as
  p50 / p99 with aggregate queries/s.

The scheduling policy (`Scheduler`) is independent of the device: `GpuExecutor` runs the
library, and tests drive the policy with a simulated executor on the CPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np

RESOLUTIONS = [(640, 360), (1280, 720), (1920, 1080), (3840, 2160)]
N_CHOICES = [4, 8, 32]


@dataclasses.dataclass
class StreamSpec:
    sid: int
    width: int
    height: int
    n_cache: int
    seed: int               # lobes (the stream's lighting) and initial weights
    scene_seed: int = -1    # shading points; streams of one resolution view the same point set

    def __post_init__(self):
        if self.scene_seed < 0:
            self.scene_seed = self.seed

    @property
    def points(self) -> int:
        return self.width * self.height


def make_stream_specs(seed: int, n_streams: int):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 77])))
    out = []
    for i in range(n_streams):
        r = int(rng.integers(len(RESOLUTIONS)))
        w, h = RESOLUTIONS[r]
        n = N_CHOICES[int(rng.integers(len(N_CHOICES)))]
        out.append(StreamSpec(i, w, h, n, seed * 1000 + i, seed * 1000 + 500 + r))
    return out


def poisson_arrivals(seed: int, rate_hz: float, duration_s: float, n_streams: int):
    """Seeded Poisson process of frame arrivals (aggregate rate), each for a uniform stream."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 78])))
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            return out
        out.append((t, int(rng.integers(n_streams))))


@dataclasses.dataclass
class Frame:
    sid: int
    index: int          # frame number within its stream
    arrival: float      # seconds since start
    done: float = math.nan


class Scheduler:
    """Admission + continuous batching policy.  `executor` provides:
         bytes_for(spec) -> int, admit(spec), release(sid), evict(sid),
         submit(frames) -> handle, poll(handle) -> completion time (s) or None, now() -> s.
    admit() of an evicted stream restores the state evict() saved."""

    def __init__(self, specs, executor, budget_bytes: int, max_batch: int = 16, max_inflight: int = 2):
        self.specs = {s.sid: s for s in specs}
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.used = 0
        self.peak_used = 0
        self.admitted = set()
        self.pending = collections.defaultdict(collections.deque)   # sid -> deque[Frame]
        self.waiting = []        # sids with frames but not admitted, in arrival order
        self.busy = set()        # sids with a frame in flight
        self.inflight = collections.deque()
        self.remaining = collections.Counter()   # frames not yet arrived, per stream
        self.done = []
        self.admit_log = []
        self.wait_since = {}     # sid -> time it started waiting for admission
        self.admit_waits = []    # (sid, seconds waited for memory)
        self.batch_sizes = []
        self.last_used = {}      # sid -> time of its last launch (eviction order)
        self.evictions = 0

    def _evict_for(self, need):
        """Evicts idle resident streams, least recently used first, until `need` bytes fit."""
        idle = [sid for sid in self.admitted if not self.pending[sid] and sid not in self.busy]
        idle.sort(key=lambda sid: self.last_used.get(sid, -1.0))
        for sid in idle:
            if self.used + need <= self.budget:
                break
            self.ex.evict(sid)
            self.used -= self.ex.bytes_for(self.specs[sid])
            self.admitted.discard(sid)
            self.evictions += 1

    def _try_admit(self):
        keep = []
        for i, sid in enumerate(self.waiting):
            need = self.ex.bytes_for(self.specs[sid])
            if need > self.budget:
                raise ValueError(f"stream {sid} needs {need} bytes, more than the whole budget")
            if i == 0 and self.used + need > self.budget:
                self._evict_for(need)   # room for the head of the queue
            if self.used + need <= self.budget:
                self.ex.admit(self.specs[sid])
                self.used += need
                self.peak_used = max(self.peak_used, self.used)
                self.admitted.add(sid)
                now = self.ex.now()
                self.admit_log.append((now, sid, self.used))
                self.admit_waits.append((sid, now - self.wait_since.pop(sid, now)))
            else:
                keep.append(sid)
        self.waiting = keep

    def _release_idle(self):
        for sid in list(self.admitted):
            if not self.pending[sid] and sid not in self.busy and self.remaining[sid] == 0:
                self.ex.release(sid)
                self.used -= self.ex.bytes_for(self.specs[sid])
                self.admitted.discard(sid)

    def _launch(self):
        ready = [sid for sid in self.admitted if self.pending[sid] and sid not in self.busy]
        if not ready:
            return False
        ready.sort(key=lambda s: self.pending[s][0].arrival)
        frames = [self.pending[sid].popleft() for sid in ready[: self.max_batch]]
        self.batch_sizes.append(len(frames))
        now = self.ex.now()
        for f in frames:
            self.busy.add(f.sid)
            self.last_used[f.sid] = now
        self.inflight.append((self.ex.submit(frames), frames))
        return True

    def run(self, arrivals, counter=None):
        """arrivals: list of (t, sid) sorted by t.  Returns the completed frames."""
        for _, sid in arrivals:
            self.remaining[sid] += 1
        nxt = collections.Counter()
        i = 0
        total = len(arrivals)
        while len(self.done) < total:
            now = self.ex.now()
            while i < total and arrivals[i][0] <= now:
                t, sid = arrivals[i]
                self.pending[sid].append(Frame(sid, nxt[sid], t))
                nxt[sid] += 1
                self.remaining[sid] -= 1
                if sid not in self.admitted and sid not in self.waiting:
                    self.waiting.append(sid)
                    self.wait_since[sid] = t
                i += 1
            self._release_idle()
            self._try_admit()
            progressed = False
            if self.inflight:
                h, frames = self.inflight[0]
                t_done = self.ex.poll(h)
                if t_done is not None:
                    self.inflight.popleft()
                    for f in frames:
                        f.done = t_done
                        self.busy.discard(f.sid)
                        self.done.append(f)
                    progressed = True
            if len(self.inflight) < self.max_inflight:
                progressed = self._launch() or progressed
            if not progressed:
                self.ex.idle(arrivals[i][0] if i < total else None)
        self._release_idle()
        return self.done


def latency_stats(frames):
    lat = np.array([f.done - f.arrival for f in frames])
    return {"frames": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat.max() * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


def latency_by_resolution(frames, specs):
    """p50 / p99 frame latency per stream resolution."""
    by = collections.defaultdict(list)
    sp = {s.sid: s for s in specs}
    for f in frames:
        by[f"{sp[f.sid].width}x{sp[f.sid].height}"].append(f)
    return {k: latency_stats(v) for k, v in sorted(by.items(), key=lambda kv: sp[kv[1][0].sid].points)}


class GpuExecutor:
    """Runs admitted streams on the GPU with the NIRC library: per-stream resident points,
    outputs, model (FP32 master + Adam + 16-bit copy) and training workspace, and one captured
    graph of a whole frame of the mix (the persistent batched estimate, then every training step
    of all the mix's streams together)."""

    def __init__(self, precision: int = 1, train_batch: int = 65536, train_steps: int = 4, width: int = 64,
                 use_graph: bool = True):
        import torch

        from . import nirc, workload as wl
        self.torch, self.nirc, self.wl = torch, nirc, wl
        self.cfg = nirc.make_config(width=width, precision=precision)
        self.width = width
        self.train_batch = train_batch
        self.train_steps = train_steps
        self.state_bytes = nirc.nirc_state_bytes(self.cfg)
        self.workspace_bytes = nirc.nirc_workspace_bytes(self.cfg, train_batch)
        self.fixed_bytes = 0
        self.streams = {}
        # two pairs of work lists (and graphs) used alternately, so that writing the next lists
        # never races the copy or the launch of the previous ones
        self.batches = [nirc.Batch(), nirc.Batch()]
        self.train_lists = [nirc.TrainBatch(train_batch), nirc.TrainBatch(train_batch)]
        self.graphs = [None, None]
        self.turn = 0
        self.use_graph = use_graph
        self.keep_final = False
        self.final = {}
        self.swapped = {}     # sid -> training state of an evicted stream (pinned host memory)
        self.restores = 0
        self.queries = 0
        self.submits = 0
        self.host_points = {}
        self.host_stream = {}
        self.ref = torch.cuda.Event(enable_timing=True)
        self.reset_clock()

    def prepare(self, specs):
        """Draws every stream's inputs on the host before serving starts (a stream's G-buffer
        and lighting arrive with it): points in pinned memory, one set per scene, so admission
        is only device allocation plus an asynchronous copy."""
        torch, wl = self.torch, self.wl
        for spec in specs:
            key = (spec.scene_seed, spec.points)
            if key not in self.host_points:
                p = wl.make_points(spec.scene_seed, spec.points)
                self.host_points[key] = torch.from_numpy(np.stack(p.arrays())).pin_memory()
            if spec.sid not in self.host_stream:
                self.host_stream[spec.sid] = (wl.make_lobes(spec.seed), wl.make_weights(spec.seed, self.width))

    def reset_clock(self):
        self.torch.cuda.synchronize()
        self.ref.record()
        self.torch.cuda.synchronize()
        self.t0 = time.perf_counter()

    def bytes_for(self, spec: StreamSpec) -> int:
        # points (7 x FP32) + F_tl output (3 x FP32) + model state + its training workspace
        return spec.points * (7 + 3) * 4 + self.state_bytes + self.workspace_bytes

    def admit(self, spec: StreamSpec):
        torch, nirc = self.torch, self.nirc
        self.prepare([spec])
        host = self.host_points[(spec.scene_seed, spec.points)]
        dev = torch.empty(host.shape, dtype=torch.float32, device="cuda")
        dev.copy_(host, non_blocking=True)
        lobes, w0 = self.host_stream[spec.sid]
        st = dict(spec=spec, points=nirc.Points(list(dev.unbind(0))), lobes=lobes,
                  model=nirc.Model(w0, cfg=self.cfg, max_batch=self.train_batch),
                  out=torch.empty((spec.points, 3), dtype=torch.float32, device="cuda"))
        saved = self.swapped.pop(spec.sid, None)
        if saved is not None:   # an evicted stream comes back with its training state
            blob = torch.empty(saved.shape, dtype=torch.uint8, device="cuda")
            blob.copy_(saved, non_blocking=True)
            st["model"].set_state(blob, sync=False)
            st["restored_from"] = blob   # kept until the stream leaves (the copy is stream-ordered)
            self.restores += 1
        self.streams[spec.sid] = st

    def evict(self, sid: int):
        """Moves an idle stream's training state to pinned host memory and frees its device
        memory (stream-ordered: the copy runs after the stream's last frame)."""
        torch = self.torch
        st = self.streams.pop(sid)
        blob = st["model"].get_state()
        host = torch.empty(blob.shape, dtype=torch.uint8).pin_memory()
        host.copy_(blob, non_blocking=True)
        self.swapped[sid] = host

    def release(self, sid: int):
        st = self.streams.pop(sid, None)
        if st is not None and self.keep_final:
            self.final[sid] = (st["model"].get_weights(), st["out"].clone())

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def idle(self, next_arrival):
        time.sleep(0.0002)

    def submit(self, frames):
        torch, nirc = self.torch, self.nirc
        reqs = []
        for f in frames:
            st = self.streams[f.sid]
            self.queries += st["spec"].points * (st["spec"].n_cache + 1)
            reqs.append(dict(model=st["model"], points=st["points"], lobes=st["lobes"].rotated(f.index).packed(),
                             n_cache=st["spec"].n_cache, seed=st["spec"].seed, frame=f.index, out_tl=st["out"]))
        treqs = [dict(model=r["model"], points=r["points"], lobes=r["lobes"], batch=self.train_batch, seed=r["seed"],
                      frame=r["frame"]) for r in reqs]
        k = self.turn
        self.turn ^= 1
        self.submits += 1
        batch, tlist = self.batches[k], self.train_lists[k]
        batch.set(reqs)
        tlist.set(treqs)
        if self.use_graph:
            if self.graphs[k] is None:
                # the first use of a pair of lists runs eagerly, then the frame is captured
                batch.launch()
                tlist.launch(self.train_steps)
                torch.cuda.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=torch.cuda.Stream()):
                    batch.launch()
                    tlist.launch(self.train_steps)
                self.graphs[k] = g
            else:
                self.graphs[k].replay()
        else:
            batch.launch()
            tlist.launch(self.train_steps)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        return ev

    def poll(self, ev):
        if not ev.query():
            return None
        return self.ref.elapsed_time(ev) * 1e-3 - 0.0   # GPU time since start (s)


def run_alone(executor: GpuExecutor, spec: StreamSpec, n_frames: int):
    """One stream's frames 0..n_frames-1 on their own (tlmc_estimate + training per frame),
    returning (final weights, last estimate)."""
    torch, nirc, wl = executor.torch, executor.nirc, executor.wl
    pts = nirc.Points.from_workload(wl.make_points(spec.scene_seed, spec.points))
    lobes = wl.make_lobes(spec.seed)
    model = nirc.Model(wl.make_weights(spec.seed, executor.width), cfg=executor.cfg, max_batch=executor.train_batch)
    out = torch.empty((spec.points, 3), dtype=torch.float32, device="cuda")
    for f in range(n_frames):
        lob = lobes.rotated(f).packed()
        nirc.tlmc_estimate(model, pts, lob, spec.n_cache, spec.seed, f, out=out)
        for s in range(executor.train_steps):   # step by step through the separate entry points
            q, tgt = nirc.tlmc_train_batch(pts, lob, executor.train_batch, spec.seed, f, s)
            nirc.nirc_train_step(model, pts, q, tgt)
    return model.get_weights(), out


def serve_run(seed: int = 5, n_streams: int = 16, rate_hz: float = 240.0, duration_s: float = 10.0,
              budget_bytes: int | None = None, precision: int = 1, train_batch: int = 65536, train_steps: int = 4,
              specs=None):
    """The multi-stream loop on the GPU; returns (stats dict, scheduler, executor)."""
    ex = GpuExecutor(precision=precision, train_batch=train_batch, train_steps=train_steps)
    specs = specs or make_stream_specs(seed, n_streams)
    arrivals = poisson_arrivals(seed, rate_hz, duration_s, len(specs))
    if budget_bytes is None:
        budget_bytes = ex.fixed_bytes + sum(ex.bytes_for(s) for s in specs)
    elif budget_bytes < 1.0:   # a fraction of what all streams would hold at once
        budget_bytes = int(ex.fixed_bytes + budget_bytes * sum(ex.bytes_for(s) for s in specs))
    sch = Scheduler(specs, ex, budget_bytes - ex.fixed_bytes)
    ex.prepare(specs)
    ex.reset_clock()
    t0 = ex.now()
    done = sch.run(arrivals)
    ex.torch.cuda.synchronize()
    makespan = max(f.done for f in done) - min(f.arrival for f in done)
    st = latency_stats(done)
    st.update({"streams": len(specs), "arrival_rate_hz": rate_hz, "duration_s": duration_s,
               "queries": ex.queries, "makespan_s": makespan, "queries_per_s": ex.queries / makespan,
               "frames_per_s": len(done) / makespan, "batches": ex.submits,
               "mean_batch": len(done) / max(ex.submits, 1),
               "peak_resident_bytes": sch.peak_used + ex.fixed_bytes, "budget_bytes": budget_bytes,
               "all_streams_bytes": ex.fixed_bytes + sum(ex.bytes_for(s) for s in specs),
               "admissions": len(sch.admit_log), "evictions": sch.evictions,
               "admission_wait_ms": {"mean": float(np.mean([w for _, w in sch.admit_waits]) * 1e3),
                                     "p99": float(np.percentile([w for _, w in sch.admit_waits], 99) * 1e3),
                                     "max": float(max(w for _, w in sch.admit_waits) * 1e3)},
               "latency_by_resolution": latency_by_resolution(done, specs),
               "host_wall_s": ex.now() - t0})
    return st, sch, ex
