"""The minimal-copy state update (offspring_update_inplace) against the oracle.

Bar: bit for bit. The rows after the update, and the particle each slot
holds, equal the oracle's definition exactly (holes in slot order take the
extra copies in particle order); hence also the multiset of rows of the
ancestor-indexed copy. Offspring come from every resampler (oracle and
library), from concentrated and adversarial patterns (holes dense where the
extras are sparse, so a block's holes draw on many source tiles), up to
P = 5 000 000 with ragged tails and row widths 1, 3, 4 and 16; invalid counts
leave the state unchanged and raise the flag; graph replays repeat the
eager result.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1202_6163_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1202_6163_amd.api as api
    return api


def say(*a):
    print(*a, flush=True)


def gpu_update(rs, off, x, want_anc=True):
    o = torch.from_numpy(np.ascontiguousarray(off, dtype=np.int32)).cuda()
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    anc = torch.full((off.size,), -5, dtype=torch.int32, device="cuda") if want_anc else None
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    rs.offspring_update_inplace(o, xd, anc=anc, status=status)
    torch.cuda.synchronize()
    return (xd.cpu().numpy(), None if anc is None else anc.cpu().numpy(), int(status.item()))


def check(rs, off, x, what):
    xo, ao, rc = oracle.offspring_update_inplace(off, x)
    xg, ag, st = gpu_update(rs, off, x)
    assert st == rc, f"{what}: status {st} vs oracle {rc}"
    assert np.array_equal(ag, ao), f"{what}: slots differ at {np.flatnonzero(ag != ao)[:5]}"
    assert np.array_equal(xg.view(np.uint32), xo.view(np.uint32)), f"{what}: rows differ"
    return xg, ag


@pytest.mark.parametrize("kind", ["metropolis", "stratified", "multinomial"])
@pytest.mark.parametrize("sigma", [1.0, 4.0])
@pytest.mark.parametrize("P,D", [(1, 3), (5, 1), (1000, 4), (1024, 16), (1025, 3), (70001, 4)])
def test_oracle_offspring(rs, kind, sigma, P, D):
    say(f"inplace: {kind} sigma={sigma} P={P} D={D}")
    lw = workloads.normal_logweights(P, sigma, 31)
    if kind == "metropolis":
        anc, _ = oracle.metropolis(lw, 32, 4, 0)
    else:
        anc, _ = getattr(oracle, kind)(lw, 4, 0)
    off, _ = oracle.ancestors_to_offspring(anc)
    x = workloads.state_rows_exact(P, D)
    xg, _ = check(rs, off, x, f"{kind} P={P} D={D}")
    ref, _ = oracle.permute_copy(anc, x)
    a = np.sort(xg.reshape(P, D).view(np.uint32), axis=0)
    b = np.sort(ref.reshape(P, D).view(np.uint32), axis=0)
    assert np.array_equal(a, b), "not the multiset of the ancestor-indexed copy"


@pytest.mark.parametrize("D", [4, 16])
def test_library_metropolis_at_2_20(rs, D):
    """The benchmarked case: the library's Metropolis ancestors (eq. (5)'s B)
    turned into offspring by the library, then updated in place."""
    P = 1 << 20
    lw_h = workloads.normal_logweights(P, 1.0, 32)
    lw = torch.from_numpy(lw_h).cuda()
    B = torch.zeros(1, dtype=torch.int32, device="cuda")
    anc = rs.resample_metropolis_adaptive(lw, 7, 0, eps=0.01, B_max=4096, B_used=B)
    off = rs.ancestors_to_offspring(anc)
    torch.cuda.synchronize()
    off_h = off.cpu().numpy()
    assert off_h.sum() == P
    x = workloads.state_rows_exact(P, D)
    check(rs, off_h, x, f"library Metropolis B={int(B.item())} D={D}")
    say(f"holes: {np.count_nonzero(off_h == 0) / P:.3f} of the slots")


@pytest.mark.parametrize("P", [(1 << 22) + 5, 5_000_000])
def test_beyond_4096_tiles(rs, P):
    # more tiles than one block's prefix holds in a single pass: multinomial
    # offspring from the oracle, rows of width 4
    say(f"inplace: multinomial P={P}")
    lw = workloads.normal_logweights(P, 2.0, 33)
    anc, _ = oracle.multinomial(lw, 6, 0)
    off, _ = oracle.ancestors_to_offspring(anc)
    check(rs, off, workloads.state_rows_exact(P, 4), f"multinomial P={P}")


@pytest.mark.parametrize("pattern", ["identity", "one_holds_all_first", "one_holds_all_last",
                                     "one_holds_all_mid", "halves", "sparse_extras",
                                     "alternating"])
@pytest.mark.parametrize("P", [4097, 300000])
def test_patterns(rs, pattern, P):
    off = np.ones(P, dtype=np.int32)
    if pattern == "one_holds_all_first":
        off[:] = 0
        off[0] = P
    elif pattern == "one_holds_all_last":
        off[:] = 0
        off[-1] = P
    elif pattern == "one_holds_all_mid":
        off[:] = 0
        off[P // 2 + 17] = P
    elif pattern == "halves":  # holes first, two copies each after
        h = P // 2
        off[:h] = 0
        off[h:] = 1
        off[h:h + h] += 1 if 2 * h <= P else 0
    elif pattern == "sparse_extras":  # a dense block of holes, extras spread thin
        holes = min(5000, P // 20)
        off[100:100 + holes] = 0
        donors = np.linspace(100 + holes, P - 1, holes).astype(np.int64)
        np.add.at(off, donors, 1)
    elif pattern == "alternating":
        off[0::2] = 2
        off[1::2] = 0
        if P % 2:
            off[-1] = 1
    assert off.sum() == P and off.min() >= 0, pattern
    x = workloads.state_rows_exact(P, 4)
    check(rs, off, x, f"{pattern} P={P}")


@pytest.mark.parametrize("bad", ["sum_low", "sum_high", "negative"])
def test_invalid_counts(rs, bad):
    P, D = 50000, 4
    off = np.ones(P, dtype=np.int32)
    if bad == "sum_low":
        off[777] = 0
    elif bad == "sum_high":
        off[777] = 2
    else:
        off[5], off[40000] = -1, 3
    x = workloads.state_rows_exact(P, D)
    xg, ag, st = gpu_update(rs, off, x)
    assert st & rs.FLAG_BAD_ANCESTOR
    assert np.array_equal(xg, x) and np.array_equal(ag, np.arange(P))


def test_without_slots_and_graph_replays(rs):
    P, D = 200003, 16
    lw = workloads.normal_logweights(P, 2.0, 33)
    anc, _ = oracle.multinomial(lw, 9, 0)
    off_h, _ = oracle.ancestors_to_offspring(anc)
    x_h = workloads.state_rows_exact(P, D)
    xo, _, _ = oracle.offspring_update_inplace(off_h, x_h)
    xg, ag, st = gpu_update(rs, off_h, x_h, want_anc=False)
    assert st == 0 and ag is None and np.array_equal(xg, xo)
    off = torch.from_numpy(off_h).cuda()
    x0 = torch.from_numpy(x_h).cuda()
    x = x0.clone()
    ws = torch.empty(int(rs.lib.rs_inplace_workspace_bytes(P)), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rs.offspring_update_inplace(off, x, ws=ws)
    for k in range(4):
        x.copy_(x0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), xo), f"replay {k}"


@pytest.mark.parametrize("D", [4, 8, 32])
def test_unaligned_rows_and_wide_rows(rs, D):
    """Rows one float past a 16-byte boundary take the scalar path; D = 8 and
    32 the vector path with more vectors per row. Same bits either way."""
    P = 70001
    lw = workloads.normal_logweights(P, 2.0, 34)
    anc, _ = oracle.stratified(lw, 3, 0)
    off_h, _ = oracle.ancestors_to_offspring(anc)
    x_h = workloads.state_rows_exact(P, D)
    xo, ao, rc = oracle.offspring_update_inplace(off_h, x_h)
    assert rc == 0
    for aligned in (True, False):
        buf = torch.zeros(P * D + 1, dtype=torch.float32, device="cuda")
        x = (buf[:P * D] if aligned else buf[1:]).view(P, D)
        x.copy_(torch.from_numpy(x_h).cuda())
        a = torch.full((P,), -5, dtype=torch.int32, device="cuda")
        rs.offspring_update_inplace(torch.from_numpy(off_h).cuda(), x, anc=a)
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy().view(np.uint32), xo.view(np.uint32)), \
            f"D={D} aligned={aligned}: rows differ"
        assert np.array_equal(a.cpu().numpy(), ao), f"D={D} aligned={aligned}: slots differ"
