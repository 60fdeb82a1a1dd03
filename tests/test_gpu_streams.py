"""Calls on different streams at the same time (the C ABI's re-entrancy).

Calls that do not share a workspace or an output may overlap on separate
streams. Bar: bit for bit. The four resamplers and their copies run as three
concurrent branches over the same weights (Metropolis with eq. (5)'s B and
its copy; stratified then systematic with the copy in their fill; multinomial
and its copy), eagerly and captured in one graph with a fork and a join,
replayed several times with other work between the replays; every output
equals the same call made alone on the default stream.
"""
import numpy as np
import pytest
import torch

from paper_1202_6163_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1202_6163_amd.api as api
    return api


def say(*a):
    print(*a, flush=True)


def outputs(P, D):
    ints = lambda: torch.full((P,), -1, dtype=torch.int32, device="cuda")  # noqa: E731
    rows = lambda: torch.full((P, D), -1.0, dtype=torch.float32, device="cuda")  # noqa: E731
    return dict(anc_m=ints(), xo_m=rows(), anc_s=ints(), off_s=ints(), xo_s=rows(),
                anc_n=ints(), xo_n=rows())


def branches(rs, lw, x, o, seed, ws, side, status):
    """The three branches: side[0] and side[1] (None: the current stream)."""
    main = torch.cuda.current_stream()
    s0, s1 = side if side else (main, main)
    if side:
        s0.wait_stream(main)
        s1.wait_stream(main)
    with torch.cuda.stream(s0):
        for kind in ("stratified", "systematic"):
            rs.resample_and_copy(kind, lw, x, seed, 0, anc=o["anc_s"], off=o["off_s"],
                                 x_out=o["xo_s"], ws=ws[1], status=status)
    with torch.cuda.stream(s1):
        rs.resample_multinomial(lw, seed, 0, anc=o["anc_n"], ws=ws[2], status=status)
        rs.permute_copy(o["anc_n"], x, x_out=o["xo_n"], status=status)
    rs.resample_metropolis_adaptive(lw, seed, 0, eps=0.01, B_max=4096, anc=o["anc_m"], ws=ws[0],
                                    status=status)
    rs.permute_copy(o["anc_m"], x, x_out=o["xo_m"], status=status)
    if side:
        main.wait_stream(s0)
        main.wait_stream(s1)


def host(o):
    return {k: v.cpu().numpy() for k, v in o.items()}


def same(a, b, what):
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), f"{what}: {k} differs"


@pytest.mark.parametrize("P", [1000, 70001, 1 << 20])
def test_concurrent_branches_equal_single_calls(rs, P):
    D = 4
    say(f"streams: P={P}")
    lw = torch.from_numpy(workloads.normal_logweights(P, 1.0, 60)).cuda()
    x = torch.from_numpy(workloads.state_rows_exact(P, D)).cuda()
    nbytes = rs.workspace_bytes(P, rs.MULTINOMIAL)
    ws = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(3)]
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref = outputs(P, D)
    branches(rs, lw, x, ref, 9, ws, None, status)
    torch.cuda.synchronize()
    ref = host(ref)
    side = (torch.cuda.Stream(), torch.cuda.Stream())
    got = outputs(P, D)
    branches(rs, lw, x, got, 9, ws, side, status)
    torch.cuda.synchronize()
    same(ref, host(got), "eager")
    # captured with the fork and the join, replayed with other work between
    got = outputs(P, D)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        branches(rs, lw, x, got, 9, ws, side, status)
    other = torch.from_numpy(workloads.normal_logweights(P, 2.0, 61)).cuda()
    for k in range(3):
        for t in got.values():
            t.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same(ref, host(got), f"replay {k}")
        rs.resample_stratified(other, k, 0, ws=ws[1])  # the workspaces in use between replays
        rs.resample_multinomial(other, k, 0, ws=ws[2])
        torch.cuda.synchronize()
    assert int(status.item()) == 0
