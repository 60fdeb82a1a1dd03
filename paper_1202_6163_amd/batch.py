"""Batched resampling executor (binding of rs_batch_plan_init / resample_batch).

A Batch holds a fixed set of instances (tensors for log-weights, ancestors and
optionally state rows), the device plan and the workspace. run() enqueues the
whole batch on the current stream and can be captured in a HIP graph; the
plan itself is built by the native library.
"""
import ctypes

import torch

from . import _lib
from ._lib import check, lib
from .api import METROPOLIS, METROPOLIS_ADAPTIVE, STRATIFIED, SYSTEMATIC, _need, _stream_handle

KINDS = {"metropolis": METROPOLIS, "metropolis_adaptive": METROPOLIS_ADAPTIVE,
         "stratified": STRATIFIED, "systematic": SYSTEMATIC}
DEFAULT_TUNING = dict(chains_per_item=1024, unroll=8, lds_max_p=8192, blocks=0)


def default_tuning():
    """The autotuned batch parameters for this device, else the defaults."""
    from . import api
    rec = api._STORED_TUNING
    if rec and "batch" in rec:
        return dict(rec["batch"])
    return dict(DEFAULT_TUNING)


class Batch:
    def __init__(self, instances, tuning=None, device=None, stream=None, async_upload=False):
        """instances: dicts with lw, anc, kind ('metropolis' |
        'metropolis_adaptive' | 'stratified' | 'systematic'), seed, instance,
        and optionally B (for 'metropolis_adaptive' the cap of eq. (5)'s
        count), eps (eq. (5)'s tolerance), x_in, x_out, status, off (offspring
        output of a stratified/systematic instance).
        With async_upload the plan goes through pinned host memory held by
        this object and the call does not wait for the device."""
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        n = len(instances)
        if n < 1:
            raise ValueError("a batch needs at least one instance")
        self.instances = list(instances)  # keeps the tensors alive
        arr = (_lib.Instance * n)()
        for k, d in enumerate(self.instances):
            lw, anc = d["lw"], d["anc"]
            _need(lw, torch.float32, "lw")
            _need(anc, torch.int32, "anc", lw.numel())
            x_in, x_out = d.get("x_in"), d.get("x_out")
            D = 0
            if x_in is not None:
                _need(x_in, torch.float32, "x_in")
                D = x_in.numel() // max(lw.numel(), 1)
                _need(x_out, torch.float32, "x_out", x_in.numel())
            st = d.get("status")
            if st is not None:
                _need(st, torch.int32, "status")
            off = d.get("off")
            if off is not None:
                _need(off, torch.int32, "off", lw.numel())
            arr[k] = _lib.Instance(lw.data_ptr(), anc.data_ptr(),
                                   off.data_ptr() if off is not None else None,
                                   x_in.data_ptr() if x_in is not None else None,
                                   x_out.data_ptr() if x_out is not None else None,
                                   st.data_ptr() if st is not None else None, lw.numel(), D,
                                   KINDS[d["kind"]], int(d.get("B", 0)), int(d["instance"]),
                                   int(d["seed"]), float(d.get("eps", 0.0)))
        self._arr = arr
        t = dict(default_tuning(), **(tuning or {}))
        self.tuning = _lib.BatchTuning(t["chains_per_item"], t["unroll"], t["lds_max_p"],
                                       t["blocks"])
        pb = lib.rs_batch_plan_bytes(arr, n, ctypes.byref(self.tuning))
        if pb == 0:
            raise _lib.ResampleError("invalid batch instances or tuning")
        wb = lib.rs_batch_workspace_bytes(arr, n)
        self.plan_dev = torch.empty(pb, dtype=torch.uint8, device=self.device)
        self.ws = torch.empty(max(wb, 256), dtype=torch.uint8, device=self.device)
        self.plan = _lib.BatchPlan()
        self.staging = (torch.empty(pb, dtype=torch.uint8, pin_memory=True) if async_upload
                        else None)
        check(lib.rs_batch_plan_init(ctypes.byref(self.plan), arr, n, ctypes.byref(self.tuning),
                                     ctypes.c_void_p(self.plan_dev.data_ptr()), pb,
                                     ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                     ctypes.c_void_p(self.staging.data_ptr())
                                     if self.staging is not None else None,
                                     _stream_handle(stream)), "rs_batch_plan_init")

    def run(self, stream=None, instance_add=0):
        """Resample every instance; instance_add is added to each instance's
        Philox instance word (e.g. the time step of a set of filters)."""
        if instance_add:
            check(lib.resample_batch_at(ctypes.byref(self.plan), int(instance_add),
                                        _stream_handle(stream)), "resample_batch_at")
        else:
            check(lib.resample_batch(ctypes.byref(self.plan), _stream_handle(stream)),
                  "resample_batch")

    def add_log_mean_weight(self, acc, stream=None):
        """acc[k] += log mean weight of instance k (stratified/systematic) from
        the last run; acc: float64 device tensor of n instances."""
        if acc.dtype != torch.float64 or acc.numel() != self.plan.n_instances or not acc.is_cuda:
            raise ValueError("acc must be a float64 device tensor with one entry per instance")
        check(lib.rs_batch_log_mean_weight(ctypes.byref(self.plan),
                                           ctypes.c_void_p(acc.data_ptr()),
                                           _stream_handle(stream)), "rs_batch_log_mean_weight")

    def iterations(self, out, stream=None):
        """out[k] = the Metropolis iterations instance k ran in the last run
        (eq. (5)'s count for 'metropolis_adaptive'); 4-byte integer device tensor."""
        if out.element_size() != 4 or out.numel() != self.plan.n_instances or not out.is_cuda:
            raise ValueError("out must be a 4-byte integer device tensor, one entry per instance")
        check(lib.rs_batch_iterations(ctypes.byref(self.plan), ctypes.c_void_p(out.data_ptr()),
                                      _stream_handle(stream)), "rs_batch_iterations")
        return out

    @property
    def particles(self):
        return sum(d["lw"].numel() for d in self.instances)
