"""GPU serving loop: Poisson arrivals at 2000 requests/s with continuous
batching on several streams; every request's ancestors and copied state equal
the same request resampled alone (bit for bit), and the latency record is
consistent."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_serving_results_equal_alone():
    import paper_1202_6163_amd.api as rs
    from paper_1202_6163_amd.serve import (GpuExecutor, device_logweights, device_state_rows,
                                           make_requests, serve, summarize)
    reqs = make_requests(rate=2000.0, duration=1.0, seed=3, p_lo=10, p_hi=16)
    ex = GpuExecutor(n_streams=3, keep_results=True)
    sched = serve(reqs, ex, budget_bytes=256 << 20, max_batch=64)
    s = summarize(sched, 1.0)
    print(s, flush=True)
    assert s["requests"] == len(reqs) and s["rejected"] == 0
    assert s["mean_batch"] > 1.0  # requests were batched together
    rng = np.random.default_rng(0)
    sample = rng.choice(len(sched.done), size=min(150, len(sched.done)), replace=False)
    for k in sample:
        r = sched.done[k]
        assert r.state["status_host"] == 0
        lw = device_logweights(r.P, r.sigma, r.seed, "cuda")
        inst = r.id & 0xFFFFFFFF
        if r.kind == "metropolis":
            anc = rs.resample_metropolis(lw, r.B, r.seed, inst)
        else:
            anc = getattr(rs, f"resample_{r.kind}")(lw, r.seed, inst)
        assert torch.equal(anc.cpu(), r.state["anc_host"]), r.id
        if r.D:
            out = rs.permute_copy(anc, device_state_rows(r.P, r.D, "cuda"))
            assert torch.equal(out.cpu().view(torch.int32), r.state["x_out_host"].view(torch.int32))
    for r in sched.done:
        assert r.t_arrival <= r.t_admit <= r.t_start <= r.t_done + 1e-3
