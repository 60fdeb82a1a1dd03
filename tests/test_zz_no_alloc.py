"""The no-allocation entry point (resample_prefix_static), called through the
C ABI: its ancestors, offspring and cumulative weights equal those of the
workspace entry points (resample_stratified / resample_systematic /
resample_multinomial) on the same inputs, bit for bit, on two calls in a
row (the second with fewer particles, so it runs on what the first left in
the library's array), and sizes beyond its array are refused before any
launch."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1202_6163_amd import workloads

pytestmark = pytest.mark.gpu

KINDS = {"stratified": 0, "systematic": 1, "multinomial": 2}


def vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def static_call(L, kind, lw, seed, inst, with_off, with_cumw):
    P = lw.numel()
    anc = torch.full((P,), -5, dtype=torch.int32, device="cuda")
    off = torch.full((P,), -5, dtype=torch.int32, device="cuda") if with_off else None
    cumw = torch.full((P,), -1.0, dtype=torch.float64, device="cuda") if with_cumw else None
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.lib.resample_prefix_static(KINDS[kind], vp(lw), vp(anc), vp(off), P, seed, inst,
                                      vp(cumw), vp(st), stream)
    assert rc == L.RS_OK, (kind, P, rc)
    return anc, off, cumw, st


def workspace_call(L, kind, lw, seed, inst, with_off, with_cumw):
    P = lw.numel()
    anc = torch.full((P,), -7, dtype=torch.int32, device="cuda")
    off = torch.full((P,), -7, dtype=torch.int32, device="cuda") if with_off else None
    cumw = torch.full((P,), -2.0, dtype=torch.float64, device="cuda") if with_cumw else None
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    nbytes = L.lib.rs_workspace_bytes(P, KINDS[kind])
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    fn = getattr(L.lib, f"resample_{kind}")
    if kind == "multinomial":
        rc = fn(vp(lw), vp(anc), P, seed, inst, vp(cumw), vp(ws), ws.numel(), vp(st), stream)
    else:
        rc = fn(vp(lw), vp(anc), vp(off), P, seed, inst, vp(cumw), vp(ws), ws.numel(), vp(st),
                stream)
    assert rc == L.RS_OK, (kind, P, rc)
    return anc, off, cumw, st


@pytest.mark.parametrize("kind", list(KINDS))
def test_static_entry_equals_workspace_entry(kind):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1202_6163_amd import _lib as L
    with_off = kind != "multinomial"
    # two calls in a row, the second smaller; then a third at the first size
    for k, (P, sigma) in enumerate(((1 << 20, 1.0), (70001, 2.0), (1 << 20, 0.5))):
        lw = torch.from_numpy(workloads.normal_logweights(P, sigma, 40 + k)).cuda()
        seed, inst = 9 + k, k
        got = static_call(L, kind, lw, seed, inst, with_off, with_cumw=(k != 1))
        want = workspace_call(L, kind, lw, seed, inst, with_off, with_cumw=(k != 1))
        torch.cuda.synchronize()
        for g, w, name in zip(got, want, ("anc", "off", "cumw", "status")):
            if w is None:
                assert g is None
                continue
            assert torch.equal(g.view(torch.int32) if g.dtype == torch.float64 else g,
                               w.view(torch.int32) if w.dtype == torch.float64 else w), \
                (kind, P, name)
        assert int(got[3].item()) == 0


def test_static_entry_refuses_sizes_beyond_its_array():
    from paper_1202_6163_amd import _lib as L
    P = 1 << 22  # the multinomial needs about 37 MB of workspace here
    assert L.lib.rs_workspace_bytes(P, 2) > L.RS_STATIC_SCRATCH_BYTES
    lw = torch.zeros(P, dtype=torch.float32, device="cuda")
    anc = torch.full((P,), -3, dtype=torch.int32, device="cuda")
    rc = L.lib.resample_prefix_static(2, vp(lw), vp(anc), None, P, 1, 0, None, None, None)
    assert rc == L.RS_EWORKSPACE
    torch.cuda.synchronize()
    assert int((anc != -3).sum().item()) == 0  # nothing was launched
    # the prefix resamplers that need no cumulative weights fit far larger sizes
    assert L.lib.rs_workspace_bytes(1 << 24, 0) <= L.RS_STATIC_SCRATCH_BYTES
