"""Serving loop for real-time resampling requests (continuous batching).

Requests (log-weights of P particles, a resampler, optional D-float state
rows) arrive over time. The scheduler admits a request when its device
footprint fits the HBM budget, keeps its weights and state resident on the
device, and at every turn packs the admitted requests that are not yet running
into one batch (the library's batched launch) on a free stream, so batches
overlap on the device while new requests keep arriving. A finished batch
releases its requests' memory, admitting the next ones.

The scheduling policy (Scheduler) is pure host logic over an executor
interface, so it is tested on the CPU with a fake executor and clock; the
GPU executor (GpuExecutor) runs batches with paper_1202_6163_amd.batch.
"""
import collections
import dataclasses
import math
import time

import numpy as np

PLAN_BYTES_PER_REQUEST = 4096


@dataclasses.dataclass
class Request:
    id: int
    t_arrival: float
    P: int
    kind: str
    D: int = 0
    B: int = 64
    seed: int = 0
    sigma: float = 1.0
    # filled in by the scheduler
    t_admit: float = math.nan
    t_start: float = math.nan
    t_done: float = math.nan
    batch: int = -1
    state: dict = dataclasses.field(default_factory=dict)


def footprint(req):
    """Device bytes a request holds while resident: log-weights, ancestors,
    state in and out, a prefix workspace and its share of the batch plan."""
    P, D = req.P, req.D
    ws = 0
    if req.kind in ("stratified", "systematic"):
        tiles = (P + 1023) // 1024
        ws = 2048 + tiles * 40 + 256 * 8
    return 8 * P + 8 * P * D + ws + PLAN_BYTES_PER_REQUEST


class Scheduler:
    """Admission by footprint and continuous batching over an executor.

    executor must provide: n_streams, submit(stream, requests) -> handle,
    poll(handle) -> bool (finished), admit(request), release(request),
    finished_time(handle) -> float.
    """

    def __init__(self, executor, budget_bytes, max_batch=256, max_batch_particles=1 << 24):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.max_batch_particles = int(max_batch_particles)
        self.used = 0
        self.waiting = collections.deque()   # arrived, not admitted
        self.ready = collections.deque()     # admitted, not started
        self.running = {}                    # stream -> (handle, [requests])
        self.done = []
        self.n_batches = 0
        self.peak_used = 0
        self.rejected = []

    def arrive(self, req):
        if footprint(req) > self.budget:
            req.state["error"] = "request larger than the device budget"
            self.rejected.append(req)
            return
        self.waiting.append(req)

    def _admit(self, now):
        while self.waiting and self.used + footprint(self.waiting[0]) <= self.budget:
            req = self.waiting.popleft()
            self.used += footprint(req)
            self.peak_used = max(self.peak_used, self.used)
            req.t_admit = now
            self.ex.admit(req)
            self.ready.append(req)

    def _retire(self):
        for s, (h, reqs) in list(self.running.items()):
            if self.ex.poll(h):
                t = self.ex.finished_time(h)
                for r in reqs:
                    r.t_done = t
                    self.ex.release(r)
                    self.used -= footprint(r)
                    self.done.append(r)
                del self.running[s]

    def step(self, now):
        """One scheduling turn at time `now`; returns the number of batches started."""
        self._retire()
        self._admit(now)
        started = 0
        for s in range(self.ex.n_streams):
            if s in self.running or not self.ready:
                continue
            batch, particles = [], 0
            while self.ready and len(batch) < self.max_batch:
                r = self.ready[0]
                if batch and particles + r.P > self.max_batch_particles:
                    break
                batch.append(self.ready.popleft())
                particles += r.P
            for r in batch:
                r.t_start = now
                r.batch = self.n_batches
            self.running[s] = (self.ex.submit(s, batch), batch)
            self.n_batches += 1
            started += 1
        return started

    def idle(self):
        return not (self.waiting or self.ready or self.running)


class GpuExecutor:
    """Runs batches on n_streams HIP streams with the library's batched launch;
    completion times come from HIP events on the device clock."""

    def __init__(self, n_streams=4, tuning=None, keep_results=False, max_single_p=1 << 20):
        import torch

        from . import api, workloads
        self.torch, self.workloads, self.api = torch, workloads, api
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(n_streams)]
        self.n_streams = n_streams
        self.tuning = tuning
        self.keep_results = keep_results
        # A batch of one request goes through the single-call entry points
        # (the same results as the batched launch, without building a plan);
        # each stream keeps a prefix workspace for up to max_single_p particles.
        self.max_single_p = int(max_single_p)
        self.single_ws = [api.workspace(self.max_single_p, api.STRATIFIED, self.dev, stream=st)
                          for st in self.streams]
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record()
        torch.cuda.synchronize()
        self.t0_host = time.perf_counter()
        self.upload = torch.cuda.Stream(self.dev)

    def now(self):
        return time.perf_counter() - self.t0_host

    def admit(self, req):
        """Make the request resident: its weights and state rows are created on
        the device (seeded), as a filter running there would hold them."""
        torch = self.torch
        st = req.state
        with torch.cuda.stream(self.upload):
            st["lw"] = device_logweights(req.P, req.sigma, req.seed, self.dev)
            st["anc"] = torch.empty(req.P, dtype=torch.int32, device=self.dev)
            st["status"] = torch.zeros(1, dtype=torch.int32, device=self.dev)
            if req.D:
                st["x_in"] = device_state_rows(req.P, req.D, self.dev)
                st["x_out"] = torch.empty((req.P, req.D), dtype=torch.float32, device=self.dev)
            st["ready"] = torch.cuda.Event()
            st["ready"].record(self.upload)

    def submit(self, s, reqs):
        from .batch import Batch
        torch = self.torch
        stream = self.streams[s]
        if len(reqs) == 1 and reqs[0].P <= self.max_single_p:
            return self._submit_single(s, reqs[0])
        insts = []
        for r in reqs:
            st = r.state
            stream.wait_event(st["ready"])
            d = dict(lw=st["lw"], anc=st["anc"], kind=r.kind, B=r.B, seed=r.seed,
                     instance=r.id & 0xFFFFFFFF, status=st["status"])
            if r.D:
                d["x_in"], d["x_out"] = st["x_in"], st["x_out"]
            insts.append(d)
        with torch.cuda.stream(stream):
            b = Batch(insts, tuning=self.tuning, stream=stream, async_upload=True)
            b.run(stream=stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        return (b, ev)

    def _submit_single(self, s, r):
        torch, api = self.torch, self.api
        stream = self.streams[s]
        st = r.state
        stream.wait_event(st["ready"])
        inst = r.id & 0xFFFFFFFF
        with torch.cuda.stream(stream):
            if r.kind == "metropolis":
                api.resample_metropolis(st["lw"], r.B, r.seed, inst, anc=st["anc"],
                                        status=st["status"])
            else:
                fn = api.resample_stratified if r.kind == "stratified" else api.resample_systematic
                fn(st["lw"], r.seed, inst, anc=st["anc"], ws=self.single_ws[s],
                   status=st["status"])
            if r.D:
                api.permute_copy(st["anc"], st["x_in"], x_out=st["x_out"], status=st["status"])
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        return (None, ev)

    def poll(self, handle):
        return handle[1].query()

    def finished_time(self, handle):
        return self.t0_event.elapsed_time(handle[1]) * 1e-3

    def release(self, req):
        st = req.state
        if self.keep_results:
            st["anc_host"] = st["anc"].cpu()
            if req.D:
                st["x_out_host"] = st["x_out"].cpu()
            st["status_host"] = int(st["status"].item())
        for k in ("lw", "anc", "x_in", "x_out", "status", "ready"):
            st.pop(k, None)


def device_logweights(P, sigma, seed, device):
    """Seeded N(0, sigma^2) log-weights drawn on the device (request payload)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.randn(int(P), generator=g, device=device, dtype=torch.float32) * float(sigma)


def device_state_rows(P, D, device):
    """State rows X[i, d] = i + d / 8 built on the device."""
    import torch
    i = torch.arange(int(P), device=device, dtype=torch.float64)[:, None]
    d = torch.arange(int(D), device=device, dtype=torch.float64)[None, :]
    return (i + d / 8.0).to(torch.float32).contiguous()


def serve(requests, executor, budget_bytes, max_batch=256, time_limit=None):
    """Replay a request stream in real time; returns the scheduler."""
    sched = Scheduler(executor, budget_bytes, max_batch=max_batch)
    reqs = sorted(requests, key=lambda r: r.t_arrival)
    i = 0
    while i < len(reqs) or not sched.idle():
        now = executor.now()
        while i < len(reqs) and reqs[i].t_arrival <= now:
            sched.arrive(reqs[i])
            i += 1
        sched.step(now)
        if time_limit is not None and now > time_limit:
            break
        if sched.running and not sched.ready and not sched.waiting:
            time.sleep(20e-6)
    return sched


def summarize(sched, duration):
    done = [r for r in sched.done]
    if not done:
        return {"requests": 0}
    lat = np.array([r.t_done - r.t_arrival for r in done])
    queue = np.array([r.t_start - r.t_arrival for r in done])
    admit = np.array([r.t_admit - r.t_arrival for r in done])
    parts = sum(r.P for r in done)
    span = max(r.t_done for r in done) - min(r.t_arrival for r in done)
    return {
        "requests": len(done), "rejected": len(sched.rejected), "batches": sched.n_batches,
        "mean_batch": len(done) / max(sched.n_batches, 1),
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "max_latency_ms": float(lat.max() * 1e3),
        "p50_queue_ms": float(np.percentile(queue, 50) * 1e3),
        "p99_queue_ms": float(np.percentile(queue, 99) * 1e3),
        "p99_admission_wait_ms": float(np.percentile(admit, 99) * 1e3),
        "particles_per_s": parts / span if span > 0 else float("nan"),
        "offered_particles_per_s": parts / duration if duration else float("nan"),
        "peak_resident_bytes": sched.peak_used,
    }


def make_requests(rate=2000.0, duration=60.0, seed=0, p_lo=10, p_hi=20, B=64):
    from . import workloads
    out = []
    for d in workloads.request_stream(rate=rate, duration=duration, seed=seed, p_lo=p_lo,
                                      p_hi=p_hi, B=B):
        out.append(Request(id=d["id"], t_arrival=d["t"], P=d["P"], kind=d["kind"], D=d["D"],
                           B=d["B"], seed=d["seed"], sigma=d["sigma"]))
    return out
