"""Python binding of the resampling library: same names as the C ABI in
include/resample.h, torch tensors in place of device pointers.

This layer only marshals arguments: it checks dtype, device and contiguity,
allocates outputs the caller did not pass, keeps a zero-initialised pooled
workspace per (device, stream), and passes data pointers and the current HIP
stream to libresample.so. Every step of the computation runs in the library's
kernels.
"""
import ctypes

import torch

from . import _lib
from ._lib import check, lib

STRATIFIED, SYSTEMATIC, MULTINOMIAL, METROPOLIS, LOG_SUM_EXP, METROPOLIS_ADAPTIVE = (
    _lib.STRATIFIED, _lib.SYSTEMATIC, _lib.MULTINOMIAL, _lib.METROPOLIS, _lib.LOG_SUM_EXP,
    _lib.METROPOLIS_ADAPTIVE)
FLAG_NAN, FLAG_POSINF, FLAG_ALL_NEGINF, FLAG_BAD_ANCESTOR, FLAG_INTERNAL = (
    _lib.FLAG_NAN, _lib.FLAG_POSINF, _lib.FLAG_ALL_NEGINF, _lib.FLAG_BAD_ANCESTOR,
    _lib.FLAG_INTERNAL)


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, name, numel=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t


_workspaces = {}


def workspace_bytes(P, kind):
    return int(lib.rs_workspace_bytes(int(P), int(kind)))


def workspace(P, kind, device=None, stream=None):
    """Pooled, zero-initialised workspace for `kind` at size P on (device, stream).

    The library leaves a workspace reusable after every call, so one buffer
    serves all calls ordered on the same stream.
    """
    return _pooled(workspace_bytes(P, kind), device, stream)


def _pooled(need, device=None, stream=None):
    """The (device, stream) pool's buffer, grown to at least `need` bytes."""
    device = torch.device(device) if device is not None else torch.device(
        "cuda", torch.cuda.current_device())
    s = stream if stream is not None else torch.cuda.current_stream(device)
    key = (device.index, s.cuda_stream)
    buf = _workspaces.get(key)
    if buf is None or buf.numel() < need:
        with torch.cuda.stream(s):
            buf = torch.zeros(max(need, 256), dtype=torch.uint8, device=device)
        _workspaces[key] = buf
    return buf


def _status_ptr(status):
    if status is None:
        return None
    _need(status, torch.int32, "status")
    return _ptr(status)


def resample_metropolis(lw, B, seed, instance=0, anc=None, status=None, stream=None):
    _need(lw, torch.float32, "lw")
    P = lw.numel()
    anc = torch.empty(P, dtype=torch.int32, device=lw.device) if anc is None else anc
    _need(anc, torch.int32, "anc", P)
    check(lib.resample_metropolis(_ptr(lw), _ptr(anc), P, int(B), int(seed), int(instance),
                                  _status_ptr(status), _stream_handle(stream)),
          "resample_metropolis")
    return anc


def resample_metropolis_adaptive(lw, seed, instance=0, eps=0.01, B_max=8192, anc=None,
                                 B_used=None, ws=None, status=None, stream=None):
    """Metropolis with B from eq. (5) for these weights, computed on the device."""
    _need(lw, torch.float32, "lw")
    P = lw.numel()
    anc = torch.empty(P, dtype=torch.int32, device=lw.device) if anc is None else anc
    _need(anc, torch.int32, "anc", P)
    if B_used is not None:
        # the C ABI writes a uint32; int32 storage reads the same (B_max < 2^31)
        if B_used.dtype not in (torch.int32, torch.uint32):
            raise TypeError(f"B_used: expected a uint32 (or int32) tensor, got {B_used.dtype}")
        _need(B_used, B_used.dtype, "B_used", 1)
        if int(B_max) >= 1 << 31:
            raise ValueError("B_max must be below 2^31")
    if ws is None:
        ws = workspace(P, _lib.METROPOLIS_ADAPTIVE, lw.device, stream)
    check(lib.resample_metropolis_adaptive(_ptr(lw), _ptr(anc), P, float(eps), int(B_max),
                                           int(seed), int(instance), _ptr(ws), ws.numel(),
                                           _ptr(B_used), _status_ptr(status),
                                           _stream_handle(stream)),
          "resample_metropolis_adaptive")
    return anc


def _prefix(fn, kind, lw, seed, instance, anc, cumw, ws, status, stream, off=None,
            with_anc=True):
    _need(lw, torch.float32, "lw")
    P = lw.numel()
    if with_anc:
        anc = torch.empty(P, dtype=torch.int32, device=lw.device) if anc is None else anc
        _need(anc, torch.int32, "anc", P)
    if off is not None:
        _need(off, torch.int32, "off", P)
    if cumw is not None:
        _need(cumw, torch.float64, "cumw", P)
    if ws is None:
        ws = workspace(P, kind, lw.device, stream)
    _need(ws, torch.uint8, "ws")
    head = (_ptr(lw), _ptr(anc)) if kind == MULTINOMIAL else (_ptr(lw), _ptr(anc), _ptr(off))
    check(fn(*head, P, int(seed), int(instance), _ptr(cumw), _ptr(ws), ws.numel(),
             _status_ptr(status), _stream_handle(stream)), fn.__name__)
    return anc


def resample_stratified(lw, seed, instance=0, anc=None, cumw=None, ws=None, status=None,
                        stream=None, off=None, with_anc=True):
    """Stratified resampling; returns the ancestors (None with with_anc=False,
    which needs off). off, if given, receives the offspring counts."""
    return _prefix(lib.resample_stratified, STRATIFIED, lw, seed, instance, anc, cumw, ws, status,
                   stream, off, with_anc)


def resample_systematic(lw, seed, instance=0, anc=None, cumw=None, ws=None, status=None,
                        stream=None, off=None, with_anc=True):
    """Systematic resampling; arguments as resample_stratified."""
    return _prefix(lib.resample_systematic, SYSTEMATIC, lw, seed, instance, anc, cumw, ws, status,
                   stream, off, with_anc)


def resample_multinomial(lw, seed, instance=0, anc=None, cumw=None, ws=None, status=None,
                         stream=None):
    return _prefix(lib.resample_multinomial, MULTINOMIAL, lw, seed, instance, anc, cumw, ws,
                   status, stream)


def resample_and_copy(kind, lw, x_in, seed, instance=0, B=0, anc=None, off=None, x_out=None,
                      ws=None, status=None, stream=None):
    """Resampler `kind` ("metropolis" with B, "stratified", "systematic",
    "multinomial") with the state copy fused in; returns (anc, x_out)."""
    code = {"metropolis": METROPOLIS, "stratified": STRATIFIED, "systematic": SYSTEMATIC,
            "multinomial": MULTINOMIAL}.get(kind, kind)
    _need(lw, torch.float32, "lw")
    _need(x_in, torch.float32, "x_in")
    P = lw.numel()
    if P == 0:
        return (torch.empty(0, dtype=torch.int32, device=lw.device) if anc is None else anc,
                torch.empty_like(x_in) if x_out is None else x_out)
    if x_in.numel() % P:
        raise ValueError("x_in must hold P rows")
    D = x_in.numel() // P
    anc = torch.empty(P, dtype=torch.int32, device=lw.device) if anc is None else anc
    _need(anc, torch.int32, "anc", P)
    if off is not None:
        _need(off, torch.int32, "off", P)
    x_out = torch.empty_like(x_in) if x_out is None else x_out
    _need(x_out, torch.float32, "x_out", x_in.numel())
    if code != METROPOLIS and ws is None:
        ws = workspace(P, code, lw.device, stream)
    if ws is not None:
        _need(ws, torch.uint8, "ws")
    check(lib.resample_and_copy(int(code), _ptr(lw), _ptr(anc), _ptr(off), P, int(B), int(seed),
                                int(instance), _ptr(x_in), _ptr(x_out), D, _ptr(ws),
                                0 if ws is None else ws.numel(), _status_ptr(status),
                                _stream_handle(stream)), "resample_and_copy")
    return anc, x_out


def rs_workspace_log_sum_exp(ws, P, out=None, stream=None):
    """log sum exp(lw) computed by the last call on workspace ws (P particles)."""
    _need(ws, torch.uint8, "ws")
    out = torch.empty(1, dtype=torch.float64, device=ws.device) if out is None else out
    _need(out, torch.float64, "out", 1)
    check(lib.rs_workspace_log_sum_exp(_ptr(ws), int(P), _ptr(out), _stream_handle(stream)),
          "rs_workspace_log_sum_exp")
    return out


def resample_sorted(kind, lw, seed, instance=0, anc=None, ws=None, status=None, stream=None):
    """Sorted-weight variant of resampler `kind` ("stratified", "systematic",
    "multinomial" or the RS code); returns the ancestors (original indices).
    Graph-capturable when ws is given."""
    code = {"stratified": STRATIFIED, "systematic": SYSTEMATIC,
            "multinomial": MULTINOMIAL}.get(kind, kind)
    _need(lw, torch.float32, "lw")
    P = lw.numel()
    anc = torch.empty(P, dtype=torch.int32, device=lw.device) if anc is None else anc
    _need(anc, torch.int32, "anc", P)
    if ws is None:
        nbytes = lib.rs_sorted_workspace_bytes(P, int(code)) if P else 0
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=lw.device)
    _need(ws, torch.uint8, "ws")
    check(lib.resample_sorted(int(code), _ptr(lw), _ptr(anc), P, int(seed), int(instance),
                              _ptr(ws), ws.numel(), _status_ptr(status), _stream_handle(stream)),
          "resample_sorted")
    return anc


def ancestors_to_offspring(anc, off=None, status=None, stream=None):
    _need(anc, torch.int32, "anc")
    P = anc.numel()
    off = torch.empty(P, dtype=torch.int32, device=anc.device) if off is None else off
    _need(off, torch.int32, "off", P)
    check(lib.ancestors_to_offspring(_ptr(anc), _ptr(off), P, _status_ptr(status),
                                     _stream_handle(stream)), "ancestors_to_offspring")
    return off


def ancestors_to_offspring_ws(anc, off=None, ws=None, status=None, stream=None):
    """Offspring counts through a workspace (no device-scope atomics); ws
    defaults to the (device, stream) pool's buffer."""
    _need(anc, torch.int32, "anc")
    P = anc.numel()
    off = torch.empty(P, dtype=torch.int32, device=anc.device) if off is None else off
    _need(off, torch.int32, "off", P)
    need = int(lib.rs_offspring_workspace_bytes(P))
    if ws is None and need > 0:
        ws = _pooled(need, anc.device, stream)
    if ws is not None:
        _need(ws, torch.uint8, "ws")
    check(lib.ancestors_to_offspring_ws(_ptr(anc), _ptr(off), P, _ptr(ws),
                                        0 if ws is None else ws.numel(), _status_ptr(status),
                                        _stream_handle(stream)), "ancestors_to_offspring_ws")
    return off


def permute_copy(anc, x_in, x_out=None, status=None, stream=None):
    _need(anc, torch.int32, "anc")
    _need(x_in, torch.float32, "x_in")
    P = anc.numel()
    if P == 0:
        return torch.empty_like(x_in) if x_out is None else x_out
    if x_in.numel() % P:
        raise ValueError("x_in must hold P rows")
    D = x_in.numel() // P
    x_out = torch.empty_like(x_in) if x_out is None else x_out
    _need(x_out, torch.float32, "x_out", x_in.numel())
    check(lib.permute_copy(_ptr(anc), _ptr(x_in), _ptr(x_out), P, D, _status_ptr(status),
                           _stream_handle(stream)), "permute_copy")
    return x_out


def offspring_update_inplace(off, x, anc=None, ws=None, status=None, stream=None):
    """Minimal-copy update of the state rows x (P x D, in place) to o_j copies
    of row j; returns (x, anc) with anc[i] the particle slot i holds."""
    _need(off, torch.int32, "off")
    _need(x, torch.float32, "x")
    P = off.numel()
    if P == 0:
        return x, anc
    if x.numel() % P:
        raise ValueError("x must hold P rows")
    D = x.numel() // P
    if anc is not None:
        _need(anc, torch.int32, "anc", P)
    if ws is None:
        ws = torch.empty(int(lib.rs_inplace_workspace_bytes(P)), dtype=torch.uint8,
                         device=x.device)
    _need(ws, torch.uint8, "ws")
    check(lib.offspring_update_inplace(_ptr(off), _ptr(x), P, D, _ptr(anc), _ptr(ws), ws.numel(),
                                       _status_ptr(status), _stream_handle(stream)),
          "offspring_update_inplace")
    return x, anc


def rs_log_sum_exp(lw, out=None, ws=None, status=None, stream=None):
    _need(lw, torch.float32, "lw")
    P = lw.numel()
    out = torch.empty(1, dtype=torch.float64, device=lw.device) if out is None else out
    _need(out, torch.float64, "out")
    if ws is None:
        ws = workspace(P, LOG_SUM_EXP, lw.device, stream)
    check(lib.rs_log_sum_exp(_ptr(lw), P, _ptr(out), _ptr(ws), ws.numel(), _status_ptr(status),
                             _stream_handle(stream)), "rs_log_sum_exp")
    return out


def rs_log_u_table(approx=None, exact=None, stream=None):
    """Both logs of the 2^23-point u grid (see include/resample.h)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    approx = torch.empty(1 << 23, dtype=torch.float32, device=dev) if approx is None else approx
    exact = torch.empty(1 << 23, dtype=torch.float32, device=dev) if exact is None else exact
    _need(approx, torch.float32, "approx", 1 << 23)
    _need(exact, torch.float32, "exact", 1 << 23)
    check(lib.rs_log_u_table(_ptr(approx), _ptr(exact), _stream_handle(stream)), "rs_log_u_table")
    return approx, exact


def rs_probe_gather(w, threads, rounds, salt=1, out=None, stream=None):
    """Random-gather probe (see include/resample.h); returns out."""
    _need(w, torch.float32, "w")
    out = torch.empty(threads, dtype=torch.float32, device=w.device) if out is None else out
    check(lib.rs_probe_gather(_ptr(w), w.numel(), int(threads), int(rounds), int(salt), _ptr(out),
                              _stream_handle(stream)), "rs_probe_gather")
    return out


def rs_probe_philox(threads, rounds, seed=1, out=None, stream=None):
    """Philox-rate probe (see include/resample.h); returns out."""
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.empty(threads, dtype=torch.int32, device=dev) if out is None else out
    check(lib.rs_probe_philox(int(seed), int(threads), int(rounds), _ptr(out),
                              _stream_handle(stream)), "rs_probe_philox")
    return out


def metropolis_B(P, w_max, eps):
    return int(lib.metropolis_B(int(P), float(w_max), float(eps)))


def rs_metropolis_set_tuning(block, unroll, lds_max_p, lanes_per_chain=0):
    t = _lib.Tuning(int(block), int(unroll), int(lds_max_p), int(lanes_per_chain))
    check(lib.rs_metropolis_set_tuning(ctypes.byref(t)), "rs_metropolis_set_tuning")


def rs_metropolis_get_tuning():
    t = _lib.Tuning()
    check(lib.rs_metropolis_get_tuning(ctypes.byref(t)), "rs_metropolis_get_tuning")
    return dict(block=t.block, unroll=t.unroll, lds_max_p=t.lds_max_p,
                lanes_per_chain=t.lanes_per_chain)


def rs_prefix_set_path(path, wait_ns=-1):
    """Form of the stratified/systematic single calls: "auto", "launches" or
    "onepass" (same results; see rs_prefix_set_path in resample.h)."""
    code = {"auto": _lib.PATH_AUTO, "launches": _lib.PATH_LAUNCHES,
            "onepass": _lib.PATH_ONEPASS}[path] if isinstance(path, str) else int(path)
    check(lib.rs_prefix_set_path(code, int(wait_ns)), "rs_prefix_set_path")


def rs_prefix_get_path():
    return {_lib.PATH_AUTO: "auto", _lib.PATH_LAUNCHES: "launches",
            _lib.PATH_ONEPASS: "onepass"}[int(lib.rs_prefix_get_path())]


def _apply_stored_tuning():
    """Launch parameters from the autotuner's table for this device, if any."""
    from . import autotune
    try:
        rec = autotune.load(torch, lib) if torch.cuda.is_available() else None
    except Exception:  # a missing or unreadable table leaves the defaults
        rec = None
    if rec and "metropolis" in rec:
        rs_metropolis_set_tuning(**rec["metropolis"])
    return rec


_STORED_TUNING = _apply_stored_tuning()


RESAMPLERS = {
    "metropolis": resample_metropolis,
    "stratified": resample_stratified,
    "systematic": resample_systematic,
    "multinomial": resample_multinomial,
}


def filter_init(x, seed, stream=None):
    """x[P, D] <- initial particles z(i, t = 0) (see include/resample.h)."""
    _need(x, torch.float32, "x")
    P, D = x.shape
    check(lib.filter_init(_ptr(x), P, D, int(seed), _stream_handle(stream)), "filter_init")
    return x


def filter_init_batch(x, K, seed, stream=None):
    """x[K P, D] <- initial particles of K filters (filter k: key seed + k)."""
    _need(x, torch.float32, "x")
    KP, D = x.shape
    if KP % K:
        raise ValueError("x must hold K P rows")
    check(lib.filter_init_batch(_ptr(x), int(K), KP // K, D, int(seed), _stream_handle(stream)),
          "filter_init_batch")
    return x


def filter_propagate_weight_batch(x_in, A, y_t, q, r, seed, t, K, x_out, lw, stream=None):
    """One step of K filters at time word t: rows of filter k use key seed + k
    and variance q[k] (float64 device tensor of K)."""
    _need(x_in, torch.float32, "x_in")
    KP, D = x_in.shape
    if KP % K:
        raise ValueError("x_in must hold K P rows")
    _need(x_out, torch.float32, "x_out", KP * D)
    _need(lw, torch.float32, "lw", KP)
    _need(A, torch.float64, "A", D * D)
    _need(y_t, torch.float32, "y_t", D)
    _need(q, torch.float64, "q", K)
    check(lib.filter_propagate_weight_batch(_ptr(x_in), _ptr(x_out), _ptr(lw), int(K), KP // K, D,
                                            _ptr(A), _ptr(y_t), _ptr(q), float(r), int(seed),
                                            int(t), _stream_handle(stream)),
          "filter_propagate_weight_batch")
    return x_out, lw


def filter_loglik(lse, P, out=None, stream=None):
    """sum_t (lse[t] - log P) on the device (float64 tensor of one element)."""
    _need(lse, torch.float64, "lse")
    out = torch.empty(1, dtype=torch.float64, device=lse.device) if out is None else out
    _need(out, torch.float64, "out", 1)
    check(lib.filter_loglik(_ptr(lse), int(lse.numel()), int(P), _ptr(out),
                            _stream_handle(stream)), "filter_loglik")
    return out


def filter_propagate_weight(x_in, A, y_t, q, r, seed, t, x_out=None, lw=None, stream=None):
    """One propagation + weighting step at time t >= 1; returns (x_out, lw)."""
    _need(x_in, torch.float32, "x_in")
    P, D = x_in.shape
    x_out = torch.empty_like(x_in) if x_out is None else x_out
    lw = torch.empty(P, dtype=torch.float32, device=x_in.device) if lw is None else lw
    _need(x_out, torch.float32, "x_out", P * D)
    _need(lw, torch.float32, "lw", P)
    _need(A, torch.float64, "A", D * D)
    _need(y_t, torch.float32, "y_t", D)
    check(lib.filter_propagate_weight(_ptr(x_in), _ptr(x_out), _ptr(lw), P, D, _ptr(A), _ptr(y_t),
                                      float(q), float(r), int(seed), int(t),
                                      _stream_handle(stream)), "filter_propagate_weight")
    return x_out, lw
