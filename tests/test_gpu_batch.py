"""GPU batched resampling: every instance of a batch equals its single call
bit for bit (ancestors and copied rows), under several tunings and across
graph replays; a sample of instances also matches the oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1202_6163_amd import workloads
from parity import explained_mismatches

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1202_6163_amd.api as api
    return api


def make_instances(n, p_lo, p_hi, D, seed, with_copy=True):
    P, sig = workloads.batch_instances(n, seed=seed, p_lo=p_lo, p_hi=p_hi)
    rng = np.random.default_rng(seed + 7)
    kinds = rng.choice(["metropolis", "metropolis_adaptive", "stratified", "systematic"], size=n)
    insts = []
    for k in range(n):
        Pk = int(P[k])
        if k == 3:
            Pk = 0  # an empty instance
        lw = torch.from_numpy(workloads.normal_logweights(Pk, sig[k], 100 + k)).cuda()
        d = dict(lw=lw, anc=torch.full((Pk,), -7, dtype=torch.int32, device="cuda"),
                 kind=str(kinds[k]), B=int(rng.integers(1, 80)), seed=1000 + k,
                 instance=k, status=torch.zeros(1, dtype=torch.int32, device="cuda"))
        if d["kind"] == "metropolis_adaptive":  # B caps eq. (5)'s count, which some reach
            d["B"], d["eps"] = int(rng.integers(1, 300)), float(rng.choice([0.01, 0.1]))
        if not d["kind"].startswith("metropolis") and k % 2 == 0:
            d["off"] = torch.full((Pk,), -7, dtype=torch.int32, device="cuda")
        if with_copy and k % 5 != 1:
            Dk = D if k % 3 else 3  # some rows of a width the vector path cannot take
            d["x_in"] = torch.from_numpy(workloads.state_rows_exact(Pk, Dk)).cuda()
            d["x_out"] = torch.zeros_like(d["x_in"])
        insts.append(d)
    return insts


def single(rs, d):
    lw = d["lw"]
    off = None
    if d["kind"] == "metropolis":
        anc = rs.resample_metropolis(lw, d["B"], d["seed"], d["instance"])
    elif d["kind"] == "metropolis_adaptive":
        anc = rs.resample_metropolis_adaptive(lw, d["seed"], d["instance"], eps=d["eps"],
                                              B_max=d["B"])
    else:
        off = torch.empty_like(d["anc"]) if "off" in d else None
        anc = getattr(rs, f"resample_{d['kind']}")(lw, d["seed"], d["instance"], off=off)
    out = rs.permute_copy(anc, d["x_in"]) if "x_in" in d else None
    return anc, out, off


def check_batch(rs, insts):
    for k, d in enumerate(insts):
        anc, out, off = single(rs, d)
        assert torch.equal(d["anc"], anc), f"instance {k} ({d['kind']}, P={d['lw'].numel()})"
        if off is not None:
            assert torch.equal(d["off"], off), f"offspring of instance {k}"
        if out is not None:
            assert torch.equal(d["x_out"].view(torch.int32), out.view(torch.int32)), k
        assert int(d["status"].item()) == 0


TUNINGS = [None, dict(chains_per_item=256, unroll=2, lds_max_p=0, blocks=7),
           dict(chains_per_item=2048, unroll=16, lds_max_p=32768, blocks=0),
           dict(chains_per_item=512, unroll=4, lds_max_p=16384, blocks=64)]


@pytest.mark.parametrize("tuning", TUNINGS)
def test_batch_equals_single_calls(rs, tuning):
    from paper_1202_6163_amd.batch import Batch
    insts = make_instances(48, 6, 14, 16, seed=1)
    b = Batch(insts, tuning=tuning)
    b.run()
    torch.cuda.synchronize()
    check_batch(rs, insts)


def test_batch_matches_oracle_sample(rs):
    from paper_1202_6163_amd.batch import Batch
    insts = make_instances(12, 8, 13, 4, seed=2)
    Batch(insts).run()
    torch.cuda.synchronize()
    for d in insts:
        lw = d["lw"].cpu().numpy()
        if lw.size == 0:
            continue
        if d["kind"] == "metropolis":
            ref, _ = oracle.metropolis(lw, d["B"], d["seed"], d["instance"])
            assert np.array_equal(d["anc"].cpu().numpy(), ref)
        elif d["kind"] == "metropolis_adaptive":
            C, _, _ = oracle.cumulative(lw)
            B = min(oracle.metropolis_B(lw.size, 1.0 / C[-1], d["eps"]), d["B"])
            ref, _ = oracle.metropolis(lw, B, d["seed"], d["instance"])
            assert np.array_equal(d["anc"].cpu().numpy(), ref)
        else:
            ref, _, C = getattr(oracle, d["kind"])(lw, d["seed"], d["instance"], want_cumw=True)
            explained_mismatches(d["kind"], d["anc"].cpu().numpy(), ref, C, d["seed"],
                                 d["instance"])


def test_batch_iterations_report_eq5(rs):
    # the B each instance ran: eq. (5)'s (capped) for adaptive instances, equal
    # to the single call's B_used and to the oracle's eq. (5)
    from paper_1202_6163_amd.batch import Batch
    insts = make_instances(40, 6, 15, 4, seed=5)
    b = Batch(insts)
    b.run()
    got = b.iterations(torch.empty(len(insts), dtype=torch.int32, device="cuda")).cpu().numpy()
    for k, d in enumerate(insts):
        P = d["lw"].numel()
        if P == 0 or not d["kind"].startswith("metropolis"):
            assert got[k] == 0, k
        elif d["kind"] == "metropolis":
            assert got[k] == d["B"], k
        else:
            Bu = torch.zeros(1, dtype=torch.int32, device="cuda")
            rs.resample_metropolis_adaptive(d["lw"], d["seed"], d["instance"], eps=d["eps"],
                                            B_max=d["B"], B_used=Bu)
            C, _, _ = oracle.cumulative(d["lw"].cpu().numpy())
            want = min(oracle.metropolis_B(P, 1.0 / C[-1], d["eps"]), d["B"])
            assert got[k] == int(Bu.item()) == want, (k, got[k], want)


def test_batch_full_workload_and_graph_replays(rs):
    # 1024 instances, P log-uniform in [2^8, 2^16], Metropolis B = 64 and
    # stratified, D = 16
    from paper_1202_6163_amd.batch import Batch
    P, sig = workloads.batch_instances(1024, seed=0)
    insts = []
    for k in range(1024):
        Pk = int(P[k])
        lw = torch.from_numpy(workloads.normal_logweights(Pk, sig[k], k)).cuda()
        insts.append(dict(lw=lw, anc=torch.empty(Pk, dtype=torch.int32, device="cuda"),
                          kind="metropolis" if k % 2 else "stratified", B=64, seed=5, instance=k,
                          x_in=torch.from_numpy(workloads.state_rows_normal(Pk, 16, k)).cuda(),
                          x_out=torch.empty((Pk, 16), dtype=torch.float32, device="cuda"),
                          status=torch.zeros(1, dtype=torch.int32, device="cuda")))
    b = Batch(insts)
    b.run()
    torch.cuda.synchronize()
    check_batch(rs, insts)
    ref = [d["anc"].clone() for d in insts]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        for d in insts:
            d["anc"].fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, d in enumerate(insts):
            assert torch.equal(d["anc"], ref[k]), (rep, k)


def test_batch_long_tables_equal_single_calls(rs):
    # instances beyond 1024 tiles: the single calls' table launch runs
    # 512-thread blocks there, the batch's table launch 256-thread blocks
    # (and beyond 4096 tiles keeps its boundaries in the workspace), with the
    # runs and scans on the first 256 threads either way: the same bits
    from paper_1202_6163_amd.batch import Batch
    specs = [("stratified", (1 << 20) + 5, 4), ("systematic", 5_000_000, 0),
             ("metropolis_adaptive", 3_000_001, 0), ("stratified", 1000, 4),
             ("systematic", (1 << 22) + 3, 4)]
    insts = []
    for k, (kind, Pk, D) in enumerate(specs):
        print(f"batch long tables: instance {k} {kind} P={Pk}", flush=True)
        lw = torch.from_numpy(workloads.normal_logweights(Pk, 1.0, 300 + k)).cuda()
        d = dict(lw=lw, anc=torch.full((Pk,), -7, dtype=torch.int32, device="cuda"), kind=kind,
                 B=64, seed=77 + k, instance=k, eps=0.01,
                 status=torch.zeros(1, dtype=torch.int32, device="cuda"))
        if kind != "metropolis_adaptive":
            d["off"] = torch.full((Pk,), -7, dtype=torch.int32, device="cuda")
        if D:
            d["x_in"] = torch.from_numpy(workloads.state_rows_exact(Pk, D)).cuda()
            d["x_out"] = torch.zeros_like(d["x_in"])
        insts.append(d)
    b = Batch(insts)
    b.run()
    torch.cuda.synchronize()
    check_batch(rs, insts)


def test_batch_instance_offset_equals_single_calls(rs):
    from paper_1202_6163_amd.batch import Batch
    insts = make_instances(16, 6, 13, 4, seed=4)
    b = Batch(insts)
    add = 12345
    b.run(instance_add=add)
    torch.cuda.synchronize()
    for k, d in enumerate(insts):
        shifted = dict(d, instance=d["instance"] + add)
        anc, out, off = single(rs, shifted)
        assert torch.equal(d["anc"], anc), f"instance {k} ({d['kind']})"
        if out is not None:
            assert torch.equal(d["x_out"].view(torch.int32), out.view(torch.int32)), k
        if off is not None:
            assert torch.equal(d["off"], off), k


def test_batch_log_mean_weight(rs):
    from paper_1202_6163_amd.batch import Batch
    insts = make_instances(10, 6, 13, 4, seed=6, with_copy=False)
    b = Batch(insts)
    b.run()
    acc = torch.zeros(len(insts), dtype=torch.float64, device="cuda")
    b.add_log_mean_weight(acc)
    torch.cuda.synchronize()
    for k, d in enumerate(insts):
        P = d["lw"].numel()
        if d["kind"] == "metropolis" or P == 0:
            assert math.isnan(float(acc[k]))
        else:
            want = float(rs.rs_log_sum_exp(d["lw"])) - math.log(P)
            # same lse bits; the device log(P) may differ from the host's in the last ulp
            assert abs(float(acc[k]) - want) <= 1e-13 * max(1.0, abs(want)), k
