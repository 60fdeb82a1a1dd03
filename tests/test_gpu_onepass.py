"""The one-launch stratified/systematic resampler against the three-launch
form and against the oracle.

The one-pass kernel exchanges the tile sums between blocks through tagged
words in the workspace (cleared by a fill kernel before each call) instead of
kernel boundaries. Bar: ancestors,
offspring, cumulative weights, rows and the status word are bit for bit
those of the three launches (same tile values, same boundary code, same
fill), on every size up to 2^20 with ragged tails, with heavy tiles
(sigma = 4), when every block computes the tiles it has not seen itself
(wait bound 0), on garbage and stale workspaces, on repeated calls with
shrinking and growing P, under graph replays, and on flagged inputs; and
against the oracle at 2^20 (ancestors identical except draws within 1e-6 of
a boundary, cumulative weights within 1e-6 relative).
"""
import numpy as np
import pytest
import torch

import oracle
from parity import ORACLE_FN, check_cumw, explained_mismatches
from paper_1202_6163_amd import workloads

pytestmark = pytest.mark.gpu

KINDS = ("stratified", "systematic")


@pytest.fixture(scope="module")
def rs():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1202_6163_amd.api as api
    return api


@pytest.fixture
def path(rs):
    saved = rs.rs_prefix_get_path()
    yield
    rs.rs_prefix_set_path(saved)


def say(*a):
    print(*a, flush=True)


def run(rs, form, kind, lw, seed, inst=0, x=None, ws=None, wait_ns=-1):
    """One call in the given form; every output as host arrays."""
    rs.rs_prefix_set_path(form, wait_ns)
    P = lw.numel()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    off = torch.full((P,), -7, dtype=torch.int32, device="cuda")
    if ws is None:
        ws = rs.workspace(P, rs.STRATIFIED, lw.device)
    if x is None:
        C = torch.full((P,), -1.0, dtype=torch.float64, device="cuda")
        anc = getattr(rs, f"resample_{kind}")(lw, seed, inst, cumw=C, ws=ws, status=status, off=off)
        out = (anc, off, C)
    else:
        xo = torch.full_like(x, -3.0)
        anc, xo = rs.resample_and_copy(kind, lw, x, seed, inst, off=off, x_out=xo, ws=ws,
                                       status=status)
        out = (anc, off, xo)
    lse = rs.rs_workspace_log_sum_exp(ws, P)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out] + [int(status.item()), float(lse.item())]


def same(a, b, what):
    for k, (u, v) in enumerate(zip(a, b)):
        if isinstance(u, np.ndarray):
            assert u.dtype == v.dtype and u.shape == v.shape, f"{what}: output {k} shape"
            assert np.array_equal(u.view(np.uint8), v.view(np.uint8)), \
                f"{what}: output {k} differs at {np.flatnonzero(u != v)[:5]}"
        elif isinstance(u, float) and np.isnan(u):
            assert np.isnan(v), f"{what}: output {k}"
        else:
            assert u == v, f"{what}: output {k}: {u} vs {v}"


SIZES = [1, 3, 1000, 1024, 1025, 2048, 4099, 65536 + 7, (1 << 18) - 1, 1 << 20,
         (1 << 20) + 1]  # past 1024 tiles the one-pass path falls back to the launches


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("sigma", [1.0, 4.0])
@pytest.mark.parametrize("P", SIZES)
def test_onepass_equals_launches(rs, path, kind, sigma, P):
    say(f"onepass vs launches: {kind} P={P} sigma={sigma}")
    lw = torch.from_numpy(workloads.normal_logweights(P, sigma, 11)).cuda()
    seed = 1000 + P % 97
    a = run(rs, "launches", kind, lw, seed, 2)
    b = run(rs, "onepass", kind, lw, seed, 2)
    same(a, b, f"{kind} P={P} sigma={sigma}")
    assert a[1].sum() == P and a[3] == 0


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("D", [1, 2, 3, 4, 16])
@pytest.mark.parametrize("P", [5, 1024, 70001, 1 << 20])
def test_onepass_copy_equals_launches(rs, path, kind, D, P):
    say(f"onepass copy vs launches: {kind} P={P} D={D}")
    lw = torch.from_numpy(workloads.normal_logweights(P, 2.0, 12)).cuda()
    x = torch.from_numpy(workloads.state_rows_exact(P, D)).cuda()
    a = run(rs, "launches", kind, lw, 77, 1, x=x)
    b = run(rs, "onepass", kind, lw, 77, 1, x=x)
    same(a, b, f"{kind} copy P={P} D={D}")


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("P", [1500, 262144 + 3, 1 << 20])
def test_onepass_without_waiting(rs, path, kind, P):
    """Wait bound 0: every block reduces the tiles it has not seen on its
    first look itself; the values and results are the same bits."""
    say(f"onepass, no wait: {kind} P={P}")
    lw = torch.from_numpy(workloads.normal_logweights(P, 4.0, 13)).cuda()
    x = torch.from_numpy(workloads.state_rows_exact(P, 4)).cuda()
    a = run(rs, "launches", kind, lw, 5, 0, x=x)
    b = run(rs, "onepass", kind, lw, 5, 0, x=x, wait_ns=0)
    same(a, b, f"{kind} P={P} wait 0")
    a = run(rs, "launches", kind, lw, 6, 0)
    b = run(rs, "onepass", kind, lw, 6, 0, wait_ns=0)
    same(a, b, f"{kind} P={P} wait 0 cumw")


@pytest.mark.parametrize("fill", [0x00, 0xFF, "random", "stale"])
def test_onepass_garbage_workspace(rs, path, fill):
    """Whatever the workspace holds before the call, only this call's words
    are taken. The first call never waits (wait bound 0), so every block takes
    whatever valid-looking words it finds on its first read: the words an
    earlier call on other weights left behind carry the same tags (a word's
    tag is its index), and only the clearing fill before each call keeps
    them out."""
    P = (1 << 20) - 5
    lw = torch.from_numpy(workloads.normal_logweights(P, 1.0, 14)).cuda()
    ref = run(rs, "launches", "stratified", lw, 9, 0)
    ws = rs.workspace(P, rs.STRATIFIED, lw.device)
    if fill == "random":
        g = torch.Generator().manual_seed(3)
        ws.copy_(torch.randint(0, 256, (ws.numel(),), dtype=torch.uint8, generator=g).cuda())
    elif fill == "stale":
        # the words an earlier call on other weights left behind
        other = torch.from_numpy(workloads.normal_logweights(P, 1.0, 15)).cuda()
        run(rs, "onepass", "stratified", other, 9, 0, ws=ws)
        snap = ws.clone()
        run(rs, "onepass", "stratified", other, 9, 0, ws=ws)
        ws.copy_(snap)
    else:
        ws.fill_(fill)
    torch.cuda.synchronize()
    for k in range(3):
        got = run(rs, "onepass", "stratified", lw, 9, 0, ws=ws, wait_ns=0 if k == 0 else -1)
        same(ref, got, f"fill {fill} call {k}")


def test_onepass_sizes_change_on_one_workspace(rs, path):
    """Calls of growing and shrinking P share one workspace, which earlier
    tests may have used for any kind of call: the words a larger call
    published, with the same tags, sit past and inside a smaller call's
    words until the clearing fill."""
    sizes = [1 << 20, 3000, 1 << 20, 4097, 700000, 1 << 20, 1]
    ws = rs.workspace(1 << 20, rs.STRATIFIED, torch.device("cuda"))
    for k, P in enumerate(sizes):
        kind = KINDS[k % 2]
        lw = torch.from_numpy(workloads.normal_logweights(P, 2.0, 20 + k)).cuda()
        ref = run(rs, "launches", kind, lw, k, 0)
        got = run(rs, "onepass", kind, lw, k, 0, ws=ws[:rs.workspace_bytes(P, rs.STRATIFIED)])
        same(ref, got, f"call {k}: {kind} P={P}")


def test_onepass_after_other_kinds_on_one_workspace(rs, path):
    """One buffer serves a multinomial call at 2^20 and one-pass stratified
    calls at small P in turn. The multinomial's tile sections cover the small
    layout's published words with its own values; the one-pass calls never
    wait (wait bound 0: every block takes whatever valid-looking words it
    finds on its first read) and must still equal the launches."""
    big = 1 << 20
    ws = torch.empty(rs.workspace_bytes(big, rs.MULTINOMIAL), dtype=torch.uint8, device="cuda")
    lw_big = torch.from_numpy(workloads.normal_logweights(big, 1.0, 40)).cuda()
    for k, P in enumerate([3000, 70001, 3000, 1025, 1 << 20]):
        say(f"onepass after multinomial: call {k} P={P}")
        rs.resample_multinomial(lw_big, k, 0, ws=ws)
        lw = torch.from_numpy(workloads.normal_logweights(P, 2.0, 41 + k)).cuda()
        ref = run(rs, "launches", "stratified", lw, k, 0)
        got = run(rs, "onepass", "stratified", lw, k, 0,
                  ws=ws[:rs.workspace_bytes(P, rs.STRATIFIED)], wait_ns=0)
        same(ref, got, f"after multinomial, call {k}: P={P}")


def test_onepass_graph_replays(rs, path):
    """A captured one-pass call replayed many times (the clearing fill is a
    kernel node, replayed with it) gives the eager result on every replay,
    with eager calls on the same workspace in between."""
    P = 1 << 20
    lw = torch.from_numpy(workloads.normal_logweights(P, 1.0, 16)).cuda()
    x = torch.from_numpy(workloads.state_rows_normal(P, 4, 1)).cuda()
    rs.rs_prefix_set_path("onepass")
    ws = rs.workspace(P, rs.STRATIFIED, lw.device)
    anc = torch.empty(P, dtype=torch.int32, device="cuda")
    off = torch.empty(P, dtype=torch.int32, device="cuda")
    xo = torch.empty_like(x)
    ref = run(rs, "onepass", "systematic", lw, 4, 3, x=x)
    rs.rs_prefix_set_path("onepass")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rs.resample_and_copy("systematic", lw, x, 4, 3, anc=anc, off=off, x_out=xo, ws=ws)
    for k in range(6):
        anc.fill_(-1)
        off.fill_(-1)
        xo.fill_(0.0)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(anc.cpu().numpy(), ref[0]), f"replay {k}: ancestors"
        assert np.array_equal(off.cpu().numpy(), ref[1]), f"replay {k}: offspring"
        assert np.array_equal(xo.cpu().numpy().view(np.uint32), ref[2].view(np.uint32))
        # an eager call on another input between replays
        other = torch.from_numpy(workloads.normal_logweights(P, 2.0, 30 + k)).cuda()
        rs.resample_stratified(other, k, 0, ws=ws)
        torch.cuda.synchronize()


@pytest.mark.parametrize("case", ["nan", "posinf", "allneginf", "some_neginf"])
def test_onepass_flagged_inputs(rs, path, case):
    P = 200000
    lw_h = workloads.normal_logweights(P, 1.0, 17)
    if case == "nan":
        lw_h[123457] = np.nan
    elif case == "posinf":
        lw_h[5] = np.inf
    elif case == "allneginf":
        lw_h[:] = -np.inf
    else:
        lw_h[::3] = -np.inf
    lw = torch.from_numpy(lw_h).cuda()
    x = torch.from_numpy(workloads.state_rows_exact(P, 4)).cuda()
    for kind in KINDS:
        a = run(rs, "launches", kind, lw, 3, 0, x=x)
        b = run(rs, "onepass", kind, lw, 3, 0, x=x)
        same(a, b, f"{kind} {case}")
        if case != "some_neginf":
            assert a[3] != 0 and np.array_equal(a[0], np.arange(P, dtype=np.int32))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("sigma", [1.0, 4.0])
def test_onepass_oracle_parity_2_20(rs, path, kind, sigma):
    """The one-pass path against the oracle at the benchmarked size, with the
    state copy the benchmark step runs."""
    P, D, seed = 1 << 20, 4, 4242
    lw_h = workloads.normal_logweights(P, sigma, 18)
    x_h = workloads.state_rows_exact(P, D)
    rs.rs_prefix_set_path("onepass")
    lw, x = torch.from_numpy(lw_h).cuda(), torch.from_numpy(x_h).cuda()
    C = torch.empty(P, dtype=torch.float64, device="cuda")
    off = torch.empty(P, dtype=torch.int32, device="cuda")
    anc = getattr(rs, f"resample_{kind}")(lw, seed, 0, cumw=C, off=off)
    anc2, xo = rs.resample_and_copy(kind, lw, x, seed, 0)
    torch.cuda.synchronize()
    a, a2, o, xo = anc.cpu().numpy(), anc2.cpu().numpy(), off.cpu().numpy(), xo.cpu().numpy()
    a_o, _ = ORACLE_FN[kind](lw_h, seed, 0)
    C_o = oracle.cumulative(lw_h)[0]
    check_cumw(C.cpu().numpy(), C_o)
    m = explained_mismatches(kind, a, a_o, C_o, seed, 0)
    say(f"onepass {kind} sigma={sigma}: {m} boundary mismatches")
    assert np.array_equal(a, a2)
    assert np.array_equal(o, oracle.ancestors_to_offspring(a)[0])
    assert np.array_equal(xo.view(np.uint32), oracle.permute_copy(a, x_h)[0].view(np.uint32))
