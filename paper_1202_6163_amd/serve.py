"""Serving loop for real-time resampling requests (continuous batching).

Requests (log-weights of P particles, a resampler, optional D-float state
rows) arrive over time. The scheduler admits a request when its device
footprint fits the HBM budget, uploads its weights and state from host memory
and keeps them resident on the device, and at every turn packs the admitted
requests that are not yet running into one batch (the library's batched
launch) on a free stream, so batches overlap on the device while new requests
keep arriving. A finished batch releases its requests' memory, admitting the
next ones. Metropolis requests take B from eq. (5) for their own weights
(computed on the device, capped), so the chains are converged whenever the
cap allows; the record counts the requests whose cap bound.

Latency is measured on one host clock: arrival, admission and start are
stamped when the server acts, completion when the server's poll first sees
the request's event done (so it includes the upload and any wait for a
stream, and overstates the device's completion by at most one poll).

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
    B: int = 64        # Metropolis: the cap of eq. (5)'s iteration count
    seed: int = 0
    sigma: float = 1.0
    slot: int = 0      # which client payload holds the request's data
    eps: float = 0.01  # eq. (5)'s tolerance
    # filled in by the scheduler
    t_admit: float = math.nan
    t_start: float = math.nan
    t_done: float = math.nan
    batch: int = -1
    state: dict = dataclasses.field(default_factory=dict)


def footprint(req):
    """Device bytes a request holds while resident: log-weights, ancestors,
    state in and out, its workspace as the library sizes it (tile partials
    and table: every kind served here has one, Metropolis for eq. (5)'s B)
    and its share of the batch plan."""
    from ._lib import METROPOLIS_ADAPTIVE, STRATIFIED, lib
    P, D = req.P, req.D
    kind = METROPOLIS_ADAPTIVE if req.kind == "metropolis" else STRATIFIED
    ws = lib.rs_workspace_bytes(P, kind) + 256
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
                r.state["batch_size"] = len(batch)
            self.running[s] = (self.ex.submit(s, batch), batch)
            self.n_batches += 1
            started += 1
        return started

    def idle(self):
        return not (self.waiting or self.ready or self.running)


class Payloads:
    """The clients' side of the request data: a few payload slots in pinned
    host memory, each holding log-weights lw = sigma_k * z of P_MAX particles
    and P_MAX x 16 state values. A request names its slot; its weights are the
    first P of the slot's and its state rows the first P * D of the slot's
    values. The server uploads them at admission."""

    def __init__(self, p_max=1 << 20, n_slots=None, pin=True):
        import torch

        from . import workloads
        self.p_max = int(p_max)
        self.n_slots = int(n_slots or workloads.SERVE_SLOTS)
        self.lw, self.x = [], []
        for k in range(self.n_slots):
            lw, x = workloads.serve_payload(k, self.p_max)
            t_lw, t_x = torch.from_numpy(lw), torch.from_numpy(x)
            self.lw.append(t_lw.pin_memory() if pin else t_lw)
            self.x.append(t_x.pin_memory() if pin else t_x)

    def host(self, req):
        """(lw[P], x[P, D] or None): host views of a request's data."""
        lw = self.lw[req.slot][:req.P]
        x = self.x[req.slot][:req.P * req.D].view(req.P, req.D) if req.D else None
        return lw, x


class GpuExecutor:
    """Runs batches on n_streams HIP streams with the library's batched launch.

    A batch of one request goes through the single-call entry points (the
    same results as the batched launch, without building a plan); with
    max_batch = 1 at the scheduler every request gets its own launches."""

    def __init__(self, n_streams=4, tuning=None, keep_results=False, max_single_p=1 << 20,
                 payloads=None):
        """keep_results: True, or a set of request ids whose outputs are
        copied to the host at release (for checking)."""
        import torch

        from . import api
        self.torch, self.api = torch, api
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(n_streams)]
        self.n_streams = n_streams
        self.tuning = tuning
        self.keep_results = keep_results
        self.payloads = payloads if payloads is not None else Payloads(max_single_p)
        # each stream keeps a workspace for single requests up to max_single_p particles
        self.max_single_p = int(max_single_p)
        self.single_ws = [api.workspace(self.max_single_p, api.STRATIFIED, self.dev, stream=st)
                          for st in self.streams]
        self.upload = torch.cuda.Stream(self.dev)
        torch.cuda.synchronize()
        self.t0_host = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0_host

    def admit(self, req):
        """Make the request resident: upload its weights and state rows from
        the client's pinned host memory (asynchronously, on the upload
        stream; the request's batch waits for that copy)."""
        torch = self.torch
        st = req.state
        lw_h, x_h = self.payloads.host(req)
        with torch.cuda.stream(self.upload):
            st["lw"] = torch.empty(req.P, dtype=torch.float32, device=self.dev)
            st["lw"].copy_(lw_h, non_blocking=True)
            st["anc"] = torch.empty(req.P, dtype=torch.int32, device=self.dev)
            st["status"] = torch.zeros(1, dtype=torch.int32, device=self.dev)
            if req.D:
                st["x_in"] = torch.empty((req.P, req.D), dtype=torch.float32, device=self.dev)
                st["x_in"].copy_(x_h, non_blocking=True)
                st["x_out"] = torch.empty((req.P, req.D), dtype=torch.float32, device=self.dev)
            if req.kind == "metropolis":
                st["B_used"] = torch.zeros(1, dtype=torch.int32, device=self.dev)
                st["B_host"] = torch.zeros(1, dtype=torch.int32, pin_memory=True)
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
            kind = "metropolis_adaptive" if r.kind == "metropolis" else r.kind
            d = dict(lw=st["lw"], anc=st["anc"], kind=kind, B=r.B, eps=r.eps, seed=r.seed,
                     instance=r.id & 0xFFFFFFFF, status=st["status"])
            if r.D:
                d["x_in"], d["x_out"] = st["x_in"], st["x_out"]
            insts.append(d)
        with torch.cuda.stream(stream):
            b = Batch(insts, tuning=self.tuning, stream=stream, async_upload=True)
            b.run(stream=stream)
            # eq. (5)'s B each Metropolis request used, to pinned host memory
            # before the completion event (read at release without a sync)
            B_all = b.iterations(torch.empty(len(reqs), dtype=torch.int32, device=self.dev),
                                 stream=stream)
            for k, r in enumerate(reqs):
                if r.kind == "metropolis":
                    r.state["B_host"].copy_(B_all[k:k + 1], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return [b, ev, None]

    def _submit_single(self, s, r):
        torch, api = self.torch, self.api
        stream = self.streams[s]
        st = r.state
        stream.wait_event(st["ready"])
        inst = r.id & 0xFFFFFFFF
        with torch.cuda.stream(stream):
            if r.kind == "metropolis":
                api.resample_metropolis_adaptive(st["lw"], r.seed, inst, eps=r.eps, B_max=r.B,
                                                 anc=st["anc"], B_used=st["B_used"],
                                                 ws=self.single_ws[s], status=st["status"])
            else:
                fn = api.resample_stratified if r.kind == "stratified" else api.resample_systematic
                fn(st["lw"], r.seed, inst, anc=st["anc"], ws=self.single_ws[s],
                   status=st["status"])
            if r.D:
                api.permute_copy(st["anc"], st["x_in"], x_out=st["x_out"], status=st["status"])
            if r.kind == "metropolis":
                st["B_host"].copy_(st["B_used"], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return [None, ev, None]

    def poll(self, handle):
        if handle[2] is None and handle[1].query():
            handle[2] = self.now()  # the server sees the batch done
        return handle[2] is not None

    def finished_time(self, handle):
        return handle[2]

    def release(self, req):
        st = req.state
        if req.kind == "metropolis":
            st["B_used_host"] = int(st["B_host"][0])  # copied before the completion event
        keep = self.keep_results
        if keep is True or (keep and req.id in keep):
            st["anc_host"] = st["anc"].cpu()
            if req.D:
                st["x_out_host"] = st["x_out"].cpu()
            st["status_host"] = int(st["status"].item())
        for k in ("lw", "anc", "x_in", "x_out", "status", "ready", "B_used", "B_host"):
            st.pop(k, None)


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
    sizes = np.array([r.state.get("batch_size", 1) for r in done])
    metro = [r for r in done if r.kind == "metropolis"]
    B_used = np.array([r.state["B_used_host"] for r in metro if "B_used_host" in r.state])
    return {
        "requests": len(done), "rejected": len(sched.rejected), "batches": sched.n_batches,
        "mean_batch": len(done) / max(sched.n_batches, 1),
        "requests_in_batches_of_2_or_more": float(np.mean(sizes >= 2)),
        "admission_waits": int(np.count_nonzero(admit > 1e-4)),
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "max_latency_ms": float(lat.max() * 1e3),
        "p50_queue_ms": float(np.percentile(queue, 50) * 1e3),
        "p99_queue_ms": float(np.percentile(queue, 99) * 1e3),
        "p99_admission_wait_ms": float(np.percentile(admit, 99) * 1e3),
        "particles_per_s": parts / span if span > 0 else float("nan"),
        "offered_particles_per_s": parts / duration if duration else float("nan"),
        "peak_resident_bytes": sched.peak_used,
        "metropolis_requests": len(metro),
        "metropolis_B_median": float(np.median(B_used)) if B_used.size else None,
        "metropolis_B_capped": int(np.count_nonzero(B_used >= np.array(
            [r.B for r in metro if "B_used_host" in r.state]))) if B_used.size else 0,
    }


def make_requests(rate=2000.0, duration=60.0, seed=0, p_lo=10, p_hi=20, B=1024, eps=0.01):
    """The request stream; B is the cap of a Metropolis request's eq. (5) count."""
    from . import workloads
    out = []
    for d in workloads.request_stream(rate=rate, duration=duration, seed=seed, p_lo=p_lo,
                                      p_hi=p_hi, B=B):
        out.append(Request(id=d["id"], t_arrival=d["t"], P=d["P"], kind=d["kind"], D=d["D"],
                           B=d["B"], seed=d["seed"], sigma=d["sigma"], slot=d["slot"], eps=eps))
    return out
