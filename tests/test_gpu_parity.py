"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Bar (written here, per output):
  - Metropolis ancestors, offspring counts and the state copy: bit-exact.
  - Cumulative weights: within 1e-6 relative of the binary64 oracle.
  - Stratified / systematic / multinomial ancestors: identical except draws
    within 1e-6 relative of a cumulative-weight boundary (counted, printed).
Sizes span several 1024-weight tiles with ragged tails, up to P = 2^20 (the
largest workload) in the launch configuration the benchmark uses.
"""
import numpy as np
import pytest
import torch

import oracle
from parity import ORACLE_FN, REPORT, check_cumw, explained_mismatches
from paper_1202_6163_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1202_6163_amd.api as api
    return api


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


# ----------------------------------------------------------------- Metropolis
def test_log_u_fast_path_premise(rs):
    approx, exact = rs.rs_log_u_table()
    a, e = host(approx), host(exact)
    ref = oracle.log_u_table()
    assert np.array_equal(e.view(np.uint32), ref.view(np.uint32)), "device binary64 log differs"
    rel = np.abs(a.astype(np.float64) - e.astype(np.float64)) / np.abs(a.astype(np.float64))
    say("hardware log: max relative error on the u grid", rel.max())
    REPORT["log_u_max_rel_error"] = float(rel.max())
    assert rel.max() <= 2.0**-20


METRO_CASES = [
    (1024, 1.0, 32, 1, 0),      # the small single-resample case
    (1, 1.0, 16, 3, 0),
    (2, 0.5, 5, 3, 7),
    (3, 2.0, 9, 4, 1),
    (1000, 4.0, 64, 5, 2),
    (4097, 0.25, 7, 6, 3),
    (16384, 1.0, 64, 7, 4),
    (65537, 2.0, 33, 8, 5),
    (40000, 1.0, 17, 9, 6),
]

TUNINGS = [
    (256, 8, 16384, 0),
    (64, 2, 0, 1),
    (1024, 16, 1 << 30, 1),
    (256, 4, 1 << 30, 4),
    (128, 8, 0, 64),
    (512, 2, 1 << 30, 16),
]


@pytest.fixture
def tuning(rs):
    saved = rs.rs_metropolis_get_tuning()
    yield
    rs.rs_metropolis_set_tuning(**saved)


@pytest.mark.parametrize("P,sigma,B,seed,inst", METRO_CASES)
def test_metropolis_bit_exact(rs, tuning, P, sigma, B, seed, inst):
    lw = workloads.normal_logweights(P, sigma, seed) if P != 1024 else workloads.small_case_logweights()
    ref, st = oracle.metropolis(lw, B, seed, inst)
    g = dev(lw)
    for t in TUNINGS:
        say("metropolis", P, sigma, B, "tuning", t)
        rs.rs_metropolis_set_tuning(*t)
        anc = host(rs.resample_metropolis(g, B, seed, inst))
        assert np.array_equal(anc, ref), f"tuning {t}: {np.count_nonzero(anc != ref)} differ"


def test_metropolis_B_zero_and_special_weights(rs):
    P = 5000
    lw = workloads.normal_logweights(P, 1.0, 3)
    assert np.array_equal(host(rs.resample_metropolis(dev(lw), 0, 1)), np.arange(P))
    lw2 = lw.copy()
    lw2[::3] = -np.inf
    lw2[7] = 3.0
    ref, _ = oracle.metropolis(lw2, 40, 2, 9)
    assert np.array_equal(host(rs.resample_metropolis(dev(lw2), 40, 2, 9)), ref)
    eq = np.full(P, 0.5, dtype=np.float32)
    ref, _ = oracle.metropolis(eq, 11, 4, 0)
    assert np.array_equal(host(rs.resample_metropolis(dev(eq), 11, 4, 0)), ref)


def test_metropolis_status_flags(rs):
    lw = np.zeros(300, dtype=np.float32)
    lw[10] = np.nan
    lw[20] = np.inf
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    anc = host(rs.resample_metropolis(dev(lw), 8, 1, status=st))
    assert int(host(st)[0]) == rs.FLAG_NAN | rs.FLAG_POSINF
    ref, fl = oracle.metropolis(lw, 8, 1)
    assert fl == rs.FLAG_NAN | rs.FLAG_POSINF
    assert np.array_equal(anc, ref)  # defined outputs agree too


@pytest.mark.parametrize("B", [32, 64, 512])
@pytest.mark.parametrize("sigma", [0.25, 1.0, 4.0])
def test_metropolis_full_size(rs, B, sigma):
    P = 1 << 20
    lw = workloads.normal_logweights(P, sigma, 0)
    say("metropolis P=2^20", sigma, B)
    anc = host(rs.resample_metropolis(dev(lw), B, 0, 0))
    if B <= 64:
        ref, _ = oracle.metropolis(lw, B, 0, 0)
        assert np.array_equal(anc, ref)
    else:
        idx = np.random.default_rng(B).choice(P, 4096, replace=False)
        idx[:2] = [0, P - 1]
        ref = oracle.metropolis_subset(lw, B, 0, 0, idx)
        assert np.array_equal(anc[idx], ref)


def test_metropolis_beyond_2_20(rs):
    # a size above the benchmark's, not a power of two: the general index
    # map (high word of r P) over five million chains, weights far beyond L2
    P, B, seed, inst = 5_000_003, 8, 11, 4
    lw = workloads.normal_logweights(P, 1.0, seed)
    say("metropolis P =", P, "B =", B)
    anc = host(rs.resample_metropolis(dev(lw), B, seed, inst))
    ref, _ = oracle.metropolis(lw, B, seed, inst)
    assert np.array_equal(anc, ref)


@pytest.mark.parametrize("P,sigma", [(1000, 0.5), (4097, 2.0), (1 << 18, 1.0)])
def test_metropolis_adaptive_B(rs, P, sigma):
    lw = workloads.normal_logweights(P, sigma, 11)
    C, _, _ = oracle.cumulative(lw)
    for eps, B_max in ((0.01, 4096), (1e-3, 64)):
        B_ref = min(oracle.metropolis_B(P, 1.0 / C[-1], eps), B_max)
        B_used = torch.zeros(1, dtype=torch.int32, device="cuda")
        anc = host(rs.resample_metropolis_adaptive(dev(lw), 3, 1, eps=eps, B_max=B_max,
                                                   B_used=B_used))
        assert int(host(B_used)[0]) == B_ref
        if P <= 4097 or B_ref <= 64:
            ref, _ = oracle.metropolis(lw, B_ref, 3, 1)
            assert np.array_equal(anc, ref)
        else:
            idx = np.arange(0, P, 97)
            assert np.array_equal(anc[idx], oracle.metropolis_subset(lw, B_ref, 3, 1, idx))


def test_metropolis_deterministic(rs):
    lw = dev(workloads.normal_logweights(1 << 18, 1.0, 5))
    a = host(rs.resample_metropolis(lw, 64, 9, 1))
    b = host(rs.resample_metropolis(lw, 64, 9, 1))
    assert np.array_equal(a, b)


# ----------------------------------------------------------------- prefix resamplers
PREFIX = ["stratified", "systematic", "multinomial"]
SORTED = ["stratified", "systematic"]  # resamplers that also write offspring


def offspring_of(anc):
    off, st = oracle.ancestors_to_offspring(np.asarray(anc, dtype=np.int32))
    assert st == 0
    return off


def check_offspring(off_g, anc_g):
    """The resampler's own offspring counts are exactly the counts of its ancestors."""
    assert np.array_equal(np.asarray(off_g), offspring_of(anc_g))
SIZES = [1, 2, 3, 9, 1023, 1024, 1025, 2048, 2049, 4097, 100003, 1 << 16]


@pytest.mark.parametrize("kind", PREFIX)
@pytest.mark.parametrize("P", SIZES)
@pytest.mark.parametrize("sigma", [0.5, 2.0])
def test_prefix_parity(rs, kind, P, sigma):
    seed, inst = P % 97 + 1, 3
    lw = workloads.normal_logweights(P, sigma, seed)
    anc_o, st_o, C_o = ORACLE_FN[kind](lw, seed, inst, want_cumw=True)
    g = dev(lw)
    C = torch.empty(P, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    anc = getattr(rs, f"resample_{kind}")(g, seed, inst, cumw=C, status=st)
    anc_g, C_g = host(anc), host(C)
    assert int(host(st)[0]) == 0
    check_cumw(C_g, C_o)
    n = explained_mismatches(kind, anc_g, anc_o, C_o, seed, inst)
    if n:
        say(f"{kind} P={P} sigma={sigma}: {n} boundary mismatches (explained)")
    # the same call without cumw gives the same ancestors
    anc2 = host(getattr(rs, f"resample_{kind}")(g, seed, inst))
    assert np.array_equal(anc2, anc_g)
    if kind in SORTED:
        # offspring in the same pass (Sec. 2: these resamplers' native output),
        # with and without the ancestors
        fn = getattr(rs, f"resample_{kind}")
        off = torch.full((P,), -1, dtype=torch.int32, device="cuda")
        anc3 = host(fn(g, seed, inst, off=off))
        assert np.array_equal(anc3, anc_g)
        check_offspring(host(off), anc_g)
        off2 = torch.full((P,), -1, dtype=torch.int32, device="cuda")
        assert fn(g, seed, inst, off=off2, with_anc=False) is None
        assert torch.equal(off, off2)


@pytest.mark.parametrize("kind", PREFIX)
@pytest.mark.parametrize("sigma", [0.25, 1.0, 4.0])
def test_prefix_full_size(rs, kind, sigma):
    P = 1 << 20
    seed, inst = 4, 0
    lw = workloads.normal_logweights(P, sigma, seed)
    say(kind, "P=2^20 sigma", sigma)
    anc_o, _, C_o = ORACLE_FN[kind](lw, seed, inst, want_cumw=True)
    C = torch.empty(P, dtype=torch.float64, device="cuda")
    off = torch.full((P,), -1, dtype=torch.int32, device="cuda") if kind in SORTED else None
    kw = {"off": off} if off is not None else {}
    anc_g = host(getattr(rs, f"resample_{kind}")(dev(lw), seed, inst, cumw=C, **kw))
    worst = check_cumw(host(C), C_o)
    n = explained_mismatches(kind, anc_g, anc_o, C_o, seed, inst)
    say(f"  cumw worst rel {worst:.2e}, boundary mismatches {n}")
    if kind != "multinomial":
        assert np.all(np.diff(anc_g) >= 0)
        check_offspring(host(off), anc_g)


@pytest.mark.parametrize("kind", SORTED)
@pytest.mark.parametrize("P", [5_000_000, (1 << 24) + 4099])
def test_prefix_long_tables(rs, kind, P):
    # beyond 1024 tiles the table launch runs 512-thread blocks over runs of
    # many tiles per thread; beyond 16384 tiles (2^24 + 4099) it keeps the
    # boundaries and counts in the workspace instead of LDS, in one block
    seed, inst = 6, 2
    lw = workloads.normal_logweights(P, 1.0, seed)
    say(kind, f"P={P} (long-run table)")
    anc_o, _, C_o = ORACLE_FN[kind](lw, seed, inst, want_cumw=True)
    C = torch.empty(P, dtype=torch.float64, device="cuda")
    off = torch.full((P,), -1, dtype=torch.int32, device="cuda")
    anc_g = host(getattr(rs, f"resample_{kind}")(dev(lw), seed, inst, cumw=C, off=off))
    check_cumw(host(C), C_o)
    explained_mismatches(kind, anc_g, anc_o, C_o, seed, inst)
    check_offspring(host(off), anc_g)


@pytest.mark.parametrize("kind", SORTED)
def test_prefix_heavy_particle_overflow_chunks(rs, kind):
    # one particle carries almost all weight: its tile owns ~P outputs and is
    # split over many fill blocks
    P = 300000
    lw = np.full(P, -40.0, dtype=np.float32)
    lw[123457] = 0.0
    lw[5] = -3.0
    anc_o, _, C_o = ORACLE_FN[kind](lw, 2, 1, want_cumw=True)
    C = torch.empty(P, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    off = torch.full((P,), -1, dtype=torch.int32, device="cuda")
    anc_g = host(getattr(rs, f"resample_{kind}")(dev(lw), 2, 1, cumw=C, status=st, off=off))
    assert int(host(st)[0]) == 0
    check_cumw(host(C), C_o)
    explained_mismatches(kind, anc_g, anc_o, C_o, 2, 1)
    # the heavy tile's offspring come from draw counts, not from one block's ancestors
    check_offspring(host(off), anc_g)
    assert int(host(off)[123457]) > P // 2


def test_multinomial_heavy_particle_guide(rs):
    # one particle carries almost all weight: its group covers almost every
    # bucket of its part's guide table, and the other parts hold next to none
    P = 300000
    lw = np.full(P, -40.0, dtype=np.float32)
    lw[123457] = 0.0
    lw[5] = -3.0
    lw[299990] = -2.0
    anc_o, _, C_o = ORACLE_FN["multinomial"](lw, 2, 1, want_cumw=True)
    C = torch.empty(P, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    anc_g = host(rs.resample_multinomial(dev(lw), 2, 1, cumw=C, status=st))
    assert int(host(st)[0]) == 0
    check_cumw(host(C), C_o)
    explained_mismatches("multinomial", anc_g, anc_o, C_o, 2, 1)
    assert np.count_nonzero(anc_g == 123457) > P // 2


@pytest.mark.parametrize("P", [(1 << 20) + 1, 3_000_001, 1 << 24])
def test_multinomial_beyond_one_line_groups(rs, P):
    # above 2^20 particles a group holds more than 16 C' (one 128-byte line):
    # each draw first bisects its group's line ends (2, 4 and 16 lines here),
    # then counts within one line; 2^24 also runs the boundary table at its
    # largest LDS size (16384 tiles)
    seed, inst = 8, 5
    lw = workloads.normal_logweights(P, 2.0, seed)
    say("multinomial P =", P)
    anc_o, _, C_o = ORACLE_FN["multinomial"](lw, seed, inst, want_cumw=True)
    C = torch.empty(P, dtype=torch.float64, device="cuda")
    anc_g = host(rs.resample_multinomial(dev(lw), seed, inst, cumw=C))
    check_cumw(host(C), C_o)
    explained_mismatches("multinomial", anc_g, anc_o, C_o, seed, inst)


# (equal-weight size, zero-weight case size, zero run, single-weight size):
# the one-block multinomial path (at most 2048 particles) and the others
EDGE_CASES = [(5000, 6000, (1024, 3072), 3000), (1500, 1800, (256, 1024), 1000)]


@pytest.mark.parametrize("kind", PREFIX)
@pytest.mark.parametrize("case", EDGE_CASES)
def test_prefix_edge_weights(rs, kind, case):
    P_eq, P_zero, (z0, z1), P_one = case
    fn = getattr(rs, f"resample_{kind}")
    # equal weights: identity for stratified / systematic
    P = P_eq
    eq = np.full(P, 1.5, dtype=np.float32)
    anc_o, _ = ORACLE_FN[kind](eq, 1, 0)
    anc_g = host(fn(dev(eq), 1, 0))
    if kind != "multinomial":
        assert np.array_equal(anc_g, np.arange(P))
    assert np.array_equal(anc_g, anc_o)
    # zero weights (-inf) inside, at the ends and filling whole tiles
    lw = workloads.normal_logweights(P_zero, 1.0, 2)
    lw[:5] = -np.inf
    lw[z0:z1] = -np.inf
    lw[-7:] = -np.inf
    anc_o, _, C_o = ORACLE_FN[kind](lw, 3, 0, want_cumw=True)
    C = torch.empty(lw.size, dtype=torch.float64, device="cuda")
    kw = {}
    if kind in SORTED:
        kw["off"] = torch.full((lw.size,), -1, dtype=torch.int32, device="cuda")
    anc_g = host(fn(dev(lw), 3, 0, cumw=C, **kw))
    check_cumw(host(C), C_o)
    explained_mismatches(kind, anc_g, anc_o, C_o, 3, 0)
    assert np.all(np.isfinite(lw[anc_g])), "a zero-weight particle was selected"
    if kw:
        check_offspring(host(kw["off"]), anc_g)
    # a single finite weight takes every draw
    one = np.full(P_one, -np.inf, dtype=np.float32)
    one[P_one - 1] = 0.25
    assert np.all(host(fn(dev(one), 1, 0)) == P_one - 1)


# sizes for the three launch structures: one block (multinomial up to two
# tiles), fused table (up to 64 tiles), separate table launch
FLAG_SIZES = [1000, 2500, 100003]


@pytest.mark.parametrize("kind", PREFIX)
@pytest.mark.parametrize("P", FLAG_SIZES)
def test_prefix_flags(rs, kind, P):
    fn = getattr(rs, f"resample_{kind}")
    for bad, flag in ((np.nan, rs.FLAG_NAN), (np.inf, rs.FLAG_POSINF)):
        lw = np.zeros(P, dtype=np.float32)
        lw[2 * P // 3] = bad
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        kw = {}
        if kind in SORTED:
            kw["off"] = torch.full((P,), -1, dtype=torch.int32, device="cuda")
        C = torch.zeros(P, dtype=torch.float64, device="cuda")
        anc = host(fn(dev(lw), 1, 0, status=st, cumw=C, **kw))
        assert int(host(st)[0]) == flag
        assert np.array_equal(anc, np.arange(P))
        assert np.all(np.isnan(host(C)))
        if kw:
            assert np.all(host(kw["off"]) == 1)
    lw = np.full(P, -np.inf, dtype=np.float32)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    anc = host(fn(dev(lw), 1, 0, status=st))
    assert int(host(st)[0]) == rs.FLAG_ALL_NEGINF
    assert np.array_equal(anc, np.arange(P))
    # the workspace is clean again: a good call right after succeeds
    lw = workloads.normal_logweights(P, 1.0, 1)
    st.zero_()
    anc = host(fn(dev(lw), 1, 0, status=st))
    assert int(host(st)[0]) == 0
    anc_o, _, C_o = ORACLE_FN[kind](lw, 1, 0, want_cumw=True)
    explained_mismatches(kind, anc, anc_o, C_o, 1, 0)


def test_prefix_deterministic_and_instances_differ(rs):
    lw = dev(workloads.normal_logweights(200000, 1.0, 8))
    for kind in PREFIX:
        fn = getattr(rs, f"resample_{kind}")
        a, b = host(fn(lw, 5, 1)), host(fn(lw, 5, 1))
        assert np.array_equal(a, b)
        c = host(fn(lw, 5, 2))
        assert not np.array_equal(a, c)


def test_boundary_only_tables_at_16384_tiles(rs):
    # 2^24 particles: the table launch's largest LDS case for the kinds that
    # need only the boundaries (log-sum-exp, adaptive B)
    P = 1 << 24
    lw = workloads.normal_logweights(P, 1.0, 5)
    say("log-sum-exp and adaptive B at P =", P)
    C, m, _ = oracle.cumulative(lw)
    ref = m + np.log(C[-1])
    got = float(host(rs.rs_log_sum_exp(dev(lw)))[0])
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))
    B_ref = min(oracle.metropolis_B(P, 1.0 / C[-1], 0.01), 4)
    B_used = torch.zeros(1, dtype=torch.int32, device="cuda")
    anc = host(rs.resample_metropolis_adaptive(dev(lw), 3, 1, eps=0.01, B_max=4, B_used=B_used))
    assert int(host(B_used)[0]) == B_ref
    ref_anc, _ = oracle.metropolis(lw, B_ref, 3, 1)
    assert np.array_equal(anc, ref_anc)


def test_log_sum_exp(rs):
    for P, sigma in ((1, 1.0), (777, 2.0), (1 << 20, 4.0)):
        lw = workloads.normal_logweights(P, sigma, 1)
        C, m, _ = oracle.cumulative(lw)
        ref = m + np.log(C[-1])
        got = float(host(rs.rs_log_sum_exp(dev(lw)))[0])
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))


# ----------------------------------------------------------------- offspring, copy
@pytest.mark.parametrize("P", [1, 63, 64, 65, 1000, 4097, 1 << 20])
def test_offspring_bit_exact(rs, P):
    rng = np.random.default_rng(P)
    for anc in (rng.integers(0, P, P).astype(np.int32), np.sort(rng.integers(0, P, P)).astype(np.int32),
                np.full(P, P // 2, dtype=np.int32)):
        ref, _ = oracle.ancestors_to_offspring(anc)
        assert np.array_equal(host(rs.ancestors_to_offspring(dev(anc))), ref)


def test_offspring_bad_ancestor(rs):
    anc = np.array([0, 1, 5, -1, 2, 2], dtype=np.int32)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    off = host(rs.ancestors_to_offspring(dev(anc), status=st))
    assert int(host(st)[0]) == rs.FLAG_BAD_ANCESTOR
    assert np.array_equal(off, [1, 1, 2, 0, 0, 1])  # -1 skipped, 5 counted


# the workspace form: bucket widths 2^12 .. 2^15, one and many buckets and
# blocks, ragged last bucket, and past 2^24 the plain conversion
@pytest.mark.parametrize("P", [1, 63, 4095, 4096, 4097, 100003, 1 << 20, (1 << 20) + 3,
                               3000001, 1 << 24, (1 << 24) + 1])
def test_offspring_ws_bit_exact(rs, P):
    rng = np.random.default_rng(P + 7)
    heavy = rng.integers(0, P, P)
    heavy[rng.random(P) < 0.6] = P // 7  # one particle takes most of the draws
    pats = {"random": rng.integers(0, P, P), "sorted": np.sort(rng.integers(0, P, P)),
            "one": np.full(P, P // 2), "last": np.full(P, P - 1),
            "few": rng.choice(np.array([0, P // 3, P - 1]), size=P), "heavy": heavy}
    for name, anc in pats.items():
        anc = anc.astype(np.int32)
        ref, _ = oracle.ancestors_to_offspring(anc)
        got = host(rs.ancestors_to_offspring_ws(dev(anc)))
        assert np.array_equal(got, ref), f"{name} P={P}: differs at {np.flatnonzero(got != ref)[:5]}"


def test_offspring_ws_bad_ancestors_and_graph_replays(rs):
    anc = np.array([0, 1, 5, -1, 2, 2], dtype=np.int32)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    off = host(rs.ancestors_to_offspring_ws(dev(anc), status=st))
    assert int(host(st)[0]) == rs.FLAG_BAD_ANCESTOR
    assert np.array_equal(off, [1, 1, 2, 0, 0, 1])  # -1 skipped, 5 counted
    P = 100003
    rng = np.random.default_rng(5)
    anc = rng.integers(0, P, P).astype(np.int32)
    anc[[7, 500, 99999]] = [-5, P, P + 10]
    st.zero_()
    got = host(rs.ancestors_to_offspring_ws(dev(anc), status=st))
    assert int(host(st)[0]) == rs.FLAG_BAD_ANCESTOR
    st2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert np.array_equal(got, host(rs.ancestors_to_offspring(dev(anc), status=st2)))
    assert int(host(st2)[0]) == rs.FLAG_BAD_ANCESTOR
    # captured once, replayed on new ancestors written in place between replays
    P = (1 << 20) + 3
    a = torch.zeros(P, dtype=torch.int32, device="cuda")
    off = torch.full((P,), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(int(rs.lib.rs_offspring_workspace_bytes(P)), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rs.ancestors_to_offspring_ws(a, off=off, ws=ws)
    for k in range(4):
        anc = np.random.default_rng(40 + k).integers(0, P >> k, P).astype(np.int32)
        a.copy_(dev(anc))
        off.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref, _ = oracle.ancestors_to_offspring(anc)
        assert np.array_equal(host(off), ref), f"replay {k}"


# every D up to 100003 particles; at the full size the D of the sweep (4) and D = 1
COPY_CASES = [(P, D) for P in (1, 5, 1023, 4096, 100003) for D in (1, 3, 4, 8, 12, 16, 32)]
COPY_CASES += [(1 << 20, 1), (1 << 20, 4), (1 << 20, 16)]


@pytest.mark.parametrize("P,D", COPY_CASES)
def test_permute_copy_bit_exact(rs, P, D):
    rng = np.random.default_rng(D)
    x = workloads.state_rows_exact(P, D)
    x[rng.integers(0, P, min(P, 10))] = np.nan  # bits, not values
    for anc in (rng.integers(0, P, P).astype(np.int32), np.sort(rng.integers(0, P, P)).astype(np.int32)):
        ref, _ = oracle.permute_copy(anc, x)
        out = host(rs.permute_copy(dev(anc), dev(x)))
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("D", [4, 16])
def test_permute_copy_bad_ancestor_and_unaligned(rs, D):
    P = 100
    x = workloads.state_rows_exact(P, D)
    anc = np.arange(P, dtype=np.int32)[::-1].copy()
    anc[7] = P
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = host(rs.permute_copy(dev(anc), dev(x), status=st))
    assert int(host(st)[0]) == rs.FLAG_BAD_ANCESTOR
    assert np.all(out[7] == 0)
    ok = np.arange(P) != 7
    assert np.array_equal(out[ok], x[anc[ok]])
    # unaligned state pointers take the scalar path
    big = dev(np.concatenate([np.zeros(1, np.float32), x.ravel()]))
    out2 = torch.empty(P * D + 1, dtype=torch.float32, device="cuda")
    anc[7] = 0
    rs.permute_copy(dev(anc), big[1:], out2[1:])
    assert np.array_equal(host(out2)[1:].reshape(P, D), x[anc])


def test_binding_rejects_bad_tensors(rs):
    from paper_1202_6163_amd._lib import ResampleError
    lw = dev(np.zeros(10, np.float32))
    with pytest.raises(TypeError):
        rs.resample_metropolis(lw.double(), 4, 1)
    with pytest.raises(ValueError):
        rs.resample_metropolis(torch.zeros(10), 4, 1)
    with pytest.raises(ValueError):
        rs.resample_stratified(dev(np.zeros((4, 4), np.float32)).t(), 1)
    ws = torch.zeros(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(ResampleError):
        rs.resample_stratified(lw, 1, ws=ws)


@pytest.mark.gpu
def test_measurement_probes_run(rs):
    w = torch.randn(4096, device="cuda")
    out = rs.rs_probe_gather(w, 512, 2, 3)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()
    o2 = rs.rs_probe_philox(512, 2, 5)
    o3 = rs.rs_probe_philox(512, 2, 5)
    torch.cuda.synchronize()
    assert torch.equal(o2, o3) and int((o2 != 0).sum()) > 400


# ----------------------------------------------------------------- sorted-weight variants
@pytest.mark.parametrize("kind", PREFIX)
@pytest.mark.parametrize("P", [1, 5, 1000, 4096, 4097, 5000, 100003, 1 << 16, (1 << 20) + 3,
                               (1 << 22) + 1])
def test_sorted_variant_parity(rs, kind, P):
    seed, inst = P % 13 + 2, 1
    lw = workloads.normal_logweights(P, 1.5, seed)
    order = oracle.sorted_order(lw)
    inv = np.empty(P, dtype=np.int64)
    inv[order] = np.arange(P)
    anc_os, st, C_o = ORACLE_FN[kind](lw[order], seed, inst, want_cumw=True)
    assert st == 0
    st_g = torch.zeros(1, dtype=torch.int32, device="cuda")
    anc_g = host(rs.resample_sorted(kind, dev(lw), seed, inst, status=st_g))
    assert int(host(st_g)[0]) == 0
    # compare in the sorted order, where the draws and boundaries live
    n = explained_mismatches(kind, inv[anc_g], anc_os, C_o, seed, inst)
    if n:
        say(f"sorted {kind} P={P}: {n} boundary mismatches (explained)")
    want, _ = oracle.sorted_variant(kind, lw, seed, inst)
    assert np.count_nonzero(anc_g != want) == n


@pytest.mark.parametrize("kind", PREFIX)
def test_sorted_variant_ties_and_flags(rs, kind):
    eq = np.full(3000, 0.5, dtype=np.float32)  # ties keep index order: same as unsorted
    assert np.array_equal(host(rs.resample_sorted(kind, dev(eq), 3, 0)),
                          oracle.sorted_variant(kind, eq, 3, 0)[0])
    signed = np.zeros(2000, dtype=np.float32)
    signed[::2] = -0.0  # -0 and +0 are equal weights
    assert np.array_equal(host(rs.resample_sorted(kind, dev(signed), 4, 0)),
                          oracle.sorted_variant(kind, signed, 4, 0)[0])
    bad = np.zeros(2000, dtype=np.float32)
    bad[77] = np.nan
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    anc = host(rs.resample_sorted(kind, dev(bad), 1, 0, status=st))
    assert int(host(st)[0]) == rs.FLAG_NAN and np.array_equal(anc, np.arange(2000))


@pytest.mark.parametrize("kind", PREFIX)
def test_sorted_variant_graph_replays(rs, kind):
    """The library's own radix sort issues no memory fills: the sorted
    variant captured in a graph repeats the eager result on every replay,
    with eager work on the same workspace in between."""
    P = 300007
    lw = dev(workloads.normal_logweights(P, 2.0, 41))
    ws = torch.empty(int(rs.lib.rs_sorted_workspace_bytes(P, rs.MULTINOMIAL)), dtype=torch.uint8,
                     device="cuda")
    want = host(rs.resample_sorted(kind, lw, 7, 2, ws=ws))
    anc = torch.empty(P, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rs.resample_sorted(kind, lw, 7, 2, anc=anc, ws=ws)
    other = dev(workloads.normal_logweights(P, 1.0, 42))
    for k in range(4):
        anc.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(anc), want), f"replay {k}"
        rs.resample_sorted(kind, other, k, 0, ws=ws)
        torch.cuda.synchronize()


# ----------------------------------------------------------------- fused resample + copy
@pytest.mark.parametrize("kind", ["metropolis"] + PREFIX)
@pytest.mark.parametrize("P,D", [(1, 4), (777, 3), (5000, 4), (100003, 8), (1 << 18, 4)])
def test_resample_and_copy_equals_separate_calls(rs, kind, P, D):
    seed, inst = 11, 4
    lw = dev(workloads.normal_logweights(P, 1.0, seed))
    x = dev(workloads.state_rows_exact(P, D))
    off = (torch.full((P,), -1, dtype=torch.int32, device="cuda")
           if kind in SORTED else None)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    anc, xo = rs.resample_and_copy(kind, lw, x, seed, inst, B=24, off=off, status=st)
    if kind == "metropolis":
        ref = rs.resample_metropolis(lw, 24, seed, inst)
    elif kind == "multinomial":
        ref = rs.resample_multinomial(lw, seed, inst)
    else:
        ref_off = torch.empty_like(off)
        ref = getattr(rs, f"resample_{kind}")(lw, seed, inst, off=ref_off)
        assert torch.equal(off, ref_off)
    assert int(host(st)[0]) == 0
    assert torch.equal(anc, ref)
    want, rc = oracle.permute_copy(host(anc), host(x))
    assert rc == 0
    assert np.array_equal(host(xo).view(np.int32), want.view(np.int32))


@pytest.mark.parametrize("kind", ["metropolis"] + PREFIX)
@pytest.mark.parametrize("D", [1, 2, 5, 32])
@pytest.mark.parametrize("P", [1025, 70001])
@pytest.mark.parametrize("aligned", [True, False])
def test_resample_and_copy_row_widths(rs, kind, D, P, aligned):
    # more row widths, and state views that are not 16-byte aligned (the
    # copy's scalar path): the rows equal the oracle's copy of the ancestors,
    # which equal the plain call's
    seed, inst = 13, 2
    lw = dev(workloads.normal_logweights(P, 1.0, seed))
    rows = workloads.state_rows_exact(P, D)
    if aligned:
        x = dev(rows)
        xo = torch.full((P, D), -1.0, dtype=torch.float32, device="cuda")
    else:  # one float past a 16-byte boundary, in and out
        buf_in = torch.zeros(P * D + 1, dtype=torch.float32, device="cuda")
        buf_in[1:].copy_(dev(rows).reshape(-1))
        x = buf_in[1:].view(P, D)
        xo = torch.full((P * D + 1,), -1.0, dtype=torch.float32, device="cuda")[1:].view(P, D)
    anc, xo = rs.resample_and_copy(kind, lw, x, seed, inst, B=24, x_out=xo)
    if kind == "metropolis":
        ref = rs.resample_metropolis(lw, 24, seed, inst)
    else:
        ref = getattr(rs, f"resample_{kind}")(lw, seed, inst)
    assert torch.equal(anc, ref)
    want, rc = oracle.permute_copy(host(anc), rows)
    assert rc == 0
    assert np.array_equal(host(xo).view(np.int32), want.view(np.int32))


@pytest.mark.parametrize("kind", ["metropolis"] + PREFIX)
@pytest.mark.parametrize("P", [1 << 20, (1 << 22) + 3])
def test_resample_and_copy_full_size_against_oracle(rs, kind, P):
    # the benchmark step's form and size: P = 2^20, D = 4, one shared
    # multinomial-sized workspace, offspring for stratified/systematic; and
    # beyond 1024 tiles (the long-run table, multi-line multinomial groups)
    D, seed, inst, B = 4, 21, 2, 32
    lw_h = workloads.normal_logweights(P, 1.0, seed)
    x_h = workloads.state_rows_exact(P, D)
    lw, x = dev(lw_h), dev(x_h)
    ws = rs.workspace(P, rs.MULTINOMIAL, lw.device)
    off = torch.full((P,), -1, dtype=torch.int32, device="cuda") if kind in SORTED else None
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    say(kind, f"resample_and_copy at P={P}")
    anc, xo = rs.resample_and_copy(kind, lw, x, seed, inst, B=B, off=off, ws=ws, status=st)
    anc_g, xo_g = host(anc), host(xo)
    assert int(host(st)[0]) == 0
    if kind == "metropolis":
        # the OpenMP build of the oracle: the same bits (its own CPU test)
        anc_o, _ = oracle.metropolis_all_cores(lw_h, B, seed, inst)
        assert np.array_equal(anc_g, anc_o)
    else:
        anc_o, _, C_o = ORACLE_FN[kind](lw_h, seed, inst, want_cumw=True)
        n = explained_mismatches(kind, anc_g, anc_o, C_o, seed, inst)
        say(f"  {n} boundary mismatches (explained)")
        if kind in SORTED:
            check_offspring(host(off), anc_g)
    # rows: the oracle's copy of the GPU's ancestors, and the oracle's own rows
    # wherever the ancestors agree
    want, rc = oracle.permute_copy(anc_g, x_h)
    assert rc == 0
    assert np.array_equal(xo_g.view(np.int32), want.view(np.int32))
    rows_o, _ = oracle.permute_copy(anc_o, x_h)
    same = anc_g == anc_o
    assert np.array_equal(xo_g[same].view(np.int32), rows_o[same].view(np.int32))


@pytest.mark.parametrize("kind", ["metropolis"] + PREFIX)
def test_resample_and_copy_small_groups_and_flags(rs, kind):
    # few particles: several lanes share a Metropolis chain and split the row
    lw = dev(workloads.normal_logweights(300, 2.0, 3))
    x = dev(workloads.state_rows_exact(300, 16))
    anc, xo = rs.resample_and_copy(kind, lw, x, 5, 0, B=200)
    want, _ = oracle.permute_copy(host(anc), host(x))
    assert np.array_equal(host(xo).view(np.int32), want.view(np.int32))
    if kind != "metropolis":
        bad = np.zeros(2000, dtype=np.float32)
        bad[3] = np.nan
        xb = dev(workloads.state_rows_exact(2000, 4))
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        anc, xo = rs.resample_and_copy(kind, dev(bad), xb, 1, 0, status=st)
        assert int(host(st)[0]) == rs.FLAG_NAN
        assert np.array_equal(host(anc), np.arange(2000)) and torch.equal(xo, xb)


# ----------------------------------------------------------------- log-sum-exp read back
@pytest.mark.parametrize("kind", PREFIX)
@pytest.mark.parametrize("P", [7, 3000, 100003])
def test_workspace_log_sum_exp_equals_reduction(rs, kind, P):
    lw = dev(workloads.normal_logweights(P, 2.0, 9))
    ref = rs.rs_log_sum_exp(lw)
    ws = rs.workspace(P, rs.MULTINOMIAL, lw.device)
    getattr(rs, f"resample_{kind}")(lw, 1, 0, ws=ws)
    got = rs.rs_workspace_log_sum_exp(ws, P)
    assert torch.equal(got, ref)
    x = dev(workloads.state_rows_exact(P, 4))
    rs.resample_and_copy(kind, lw, x, 2, 0, ws=ws)
    assert torch.equal(rs.rs_workspace_log_sum_exp(ws, P), ref)
    for bad, want in ((np.nan, np.nan), (-np.inf, -np.inf)):
        b = np.full(P, bad, dtype=np.float32) if bad == -np.inf else np.zeros(P, np.float32)
        if bad != -np.inf:
            b[P // 2] = bad
        getattr(rs, f"resample_{kind}")(dev(b), 1, 0, ws=ws)
        v = float(host(rs.rs_workspace_log_sum_exp(ws, P))[0])
        assert (np.isnan(v) if np.isnan(want) else v == want), (bad, v)
