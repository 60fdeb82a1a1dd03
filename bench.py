"""Benchmark of the resampling stage on one MI355X.

Step (the timed unit): one pass of the whole resampling path over one batch
of P = 2^20 particles with log-weights N(0, sigma^2) (sigma = 1) and D = 4
binary32 state rows: the Metropolis resampler with B from eq. (5) (eps =
0.01, computed on the device from the weights, so every chain is converged
by the paper's criterion), the stratified, systematic and multinomial
resamplers, each in the paper's output form (offspring for stratified and
systematic, written in the same pass as the ancestors the copy needs;
ancestors for the other two) and the ancestor-indexed state copy (in the
stratified and systematic fill itself, a launch of its own after the other
two). Every step uses the next of many rotating input/output buffer sets
whose total exceeds the 256 MB Infinity Cache, so the step reads its inputs
from HBM. value = resampled particles per second (4 P per step) at the p99
step time.

The LAST line on stdout is a compact JSON headline (a few KB): value,
per-step times, the dominant kernel's roofline, the scan + copy path against
HBM, the CPU baseline with its parity check, and short summaries of the
other sections. The full results go to --out (default
results/bench_full.json):
  per_call      cold per-call times of every call family, with the bytes
                each timing graph touches (all above the Infinity Cache);
  step_fixed_B  the same step with Metropolis at a fixed B (flagged when B
                is below eq. (5)'s);
  roofline      the dominant kernel of the step against its ceiling;
  roofline_hbm  the stratified resample + state copy path against HBM (also
                in the one-launch form, and at 2^22 and 2^24);
  sweep         per sigma and P, p50/p99 particles/s of every resampler
                (Metropolis at each B), with and without the copy, the
                accuracy metric sum_i (o_i/P - w_i/W)^2, the ESS, eq. (5)'s B
                and the Metropolis-vs-stratified crossover (warm cache);
  dirichlet     Sec. 3's experiment: Dirichlet weights, P = 256 .. 65536,
                error and per-call time of every resampler and the
                sorted-weight variants;
  batched       1024 independent instances in one batched launch against
                per-instance calls;
  minimal_copy  the state update after Metropolis: the ancestor-indexed copy
                against the in-place minimal-copy update (D = 4 and 16);
  filter        the bootstrap filter (P = 2^18, D = 8, T = 200) against the
                Kalman log-likelihood;
  pmcmc         particle marginal Metropolis-Hastings with batched filters;
  serving       Poisson arrivals at 2000 req/s, and small requests at 8000
                and 16000 req/s batched and with per-request launches:
                latency percentiles and particles/s;
  cpu_baseline  the CPU oracle on a bounded sample of the same step (one
                pinned core, and all cores), with the GPU's outputs on the
                same inputs compared against it.
"""
import argparse
import hashlib
import math
import re
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# L2 request issue rate from the unit counts: 8 XCDs x 16 L2 channels, one
# 128-byte request per channel per clock, at 2.4 GHz.
L2_PEAK_GREQ_S = 8 * 16 * 2.4
# VALU issue rate from the unit counts: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
# Algorithmic VALU slots per Metropolis iteration: half a Philox4x32-10 block
# (10 rounds x (two quarter-rate 32x32->64 multiplies + two 3-input xors)
# / 2 = 50) plus the quarter-rate high-word multiply of the index map (4).
METRO_SLOTS_PER_ITER = 54.0
EPS = 0.01        # eq. (5) tolerance of the adaptive Metropolis leg
B_MAX = 4096      # cap of the adaptive iteration count
COLD_BYTES = 512 << 20  # every cold timing graph touches at least this much
MALL_BYTES = 256 << 20
L1_BYTES = 32 << 10  # a CU's vector L1


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--P", type=int, default=1 << 20)
    ap.add_argument("--D", type=int, default=4)
    ap.add_argument("--sigma", type=float, default=1.0)
    ap.add_argument("--B", type=int, default=32, help="fixed B of the secondary step")
    ap.add_argument("--sets", type=int, default=0,
                    help="rotating (lw, anc, off) buffer sets (0: enough for 512 MiB)")
    ap.add_argument("--reps", type=int, default=40, help="timed calls per sweep point")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--sweep-P", type=str, default="12,14,16,18,20")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-filter", action="store_true")
    ap.add_argument("--no-dirichlet", action="store_true")
    ap.add_argument("--dirichlet-R", type=int, default=50)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="seconds of Poisson arrivals at 2000 req/s (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only", type=str, default="", help="time one kernel (for profiling)")
    ap.add_argument("--out", type=str, default=os.path.join("results", "bench_full.json"))
    ap.add_argument("--record-traffic", type=str, default="",
                    help="write profiles/traffic.json from the rocprofv3 counter runs under "
                         "this directory (subdirectories <family>_<COUNTER>) and exit")
    return ap.parse_args()


from paper_1202_6163_amd.timing import Graphs, pct  # noqa: E402


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_sets(torch, workloads, P, D, n_sets, dev):
    """Rotating buffer sets: n_sets of (lw, anc, off) and enough state pairs
    (x, xo) that each kind of buffer adds up to COLD_BYTES; set k uses state
    pair k mod n_x. A graph that walks the sets re-touches a buffer only after
    more than the Infinity Cache's worth of other data."""
    n_x = max(2, -(-COLD_BYTES // (8 * P * D)))
    xs = []
    for k in range(n_x):
        x = torch.from_numpy(workloads.state_rows_normal(P, D, k)).to(dev)
        xs.append((x, torch.empty_like(x)))
    sets = []
    for s in range(n_sets):
        lw = torch.from_numpy(workloads.normal_logweights(P, SIGMA_OF_SETS, s)).to(dev)
        x, xo = xs[s % n_x]
        sets.append(dict(lw=lw, x=x, xo=xo, anc=torch.empty(P, dtype=torch.int32, device=dev),
                         off=torch.empty(P, dtype=torch.int32, device=dev)))
    return sets, n_x


SIGMA_OF_SETS = 1.0


def main():
    args = parse()
    if args.record_traffic:
        record_traffic(args.record_traffic)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU sharding is "
                                   "a design only, not built", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1202_6163_amd.api as rs
    from paper_1202_6163_amd import workloads

    global SIGMA_OF_SETS
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    P, D, sigma = args.P, args.D, args.sigma
    SIGMA_OF_SETS = sigma
    dev = torch.device("cuda", 0)
    t_start = time.perf_counter()

    n_sets = args.sets or max(8, -(-COLD_BYTES // (12 * P)))
    sets, n_x = make_sets(torch, workloads, P, D, n_sets, dev)
    ws = rs.workspace(P, rs.MULTINOMIAL, dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    B_used = torch.zeros(1, dtype=torch.int32, device=dev)
    log(f"bench: P={P} D={D} sigma={sigma}: {n_sets} (lw, anc, off) sets, {n_x} state pairs")

    # eq. (5)'s B for set 0 (the device computes it from the weights)
    rs.resample_metropolis_adaptive(sets[0]["lw"], 1, 0, eps=EPS, B_max=B_MAX,
                                    anc=sets[0]["anc"], B_used=B_used, ws=ws, status=status)
    B_eq5 = int(B_used.item())

    def step(bs, seed, inst, B=None):
        # Each resampler in the paper's output form (Sec. 2: stratified and
        # systematic give offspring, multinomial and Metropolis ancestors),
        # and the ancestor-indexed state copy. Metropolis takes eq. (5)'s B
        # for the weights at hand (B=None) or a fixed B. Stratified and
        # systematic copy the rows in their own fill (resample_and_copy);
        # Metropolis and multinomial run the copy as its own launch, which is
        # faster for them (both forms are timed and reported).
        if B is None:
            rs.resample_metropolis_adaptive(bs["lw"], seed, inst, eps=EPS, B_max=B_MAX,
                                            anc=bs["anc"], B_used=B_used, ws=ws, status=status)
        else:
            rs.resample_metropolis(bs["lw"], B, seed, inst, anc=bs["anc"], status=status)
        rs.permute_copy(bs["anc"], bs["x"], x_out=bs["xo"], status=status)
        for kind in ("stratified", "systematic"):
            rs.resample_and_copy(kind, bs["lw"], bs["x"], seed, inst, anc=bs["anc"],
                                 off=bs["off"], x_out=bs["xo"], ws=ws, status=status)
        rs.resample_multinomial(bs["lw"], seed, inst, anc=bs["anc"], ws=ws, status=status)
        rs.permute_copy(bs["anc"], bs["x"], x_out=bs["xo"], status=status)

    families = call_families(rs, ws, B_eq5, args.B)
    if args.only:
        profile_only(torch, rs, args, sets, families, step)
        return

    G = Graphs(torch)
    # ------------------------------------------------ timed steps (cold)
    step_graphs = [G.capture(lambda bs=bs, k=k: step(bs, 1000 + k, 0)) for k, bs in enumerate(sets)]
    G.replay_ms(step_graphs, max(args.warmup, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms = G.replay_ms(step_graphs, args.steps)
    wall = time.perf_counter() - t0
    assert int(status.item()) == 0, f"status flags {int(status.item())}"
    p99 = pct(step_ms, 99)
    value = 4 * P / (p99 * 1e-3)
    log(f"bench: step p50 {pct(step_ms, 50):.3f} ms p99 {p99:.3f} ms ({value:.3e} particles/s)")

    fixed_graphs = [G.capture(lambda bs=bs, k=k: step(bs, 3000 + k, 0, B=args.B))
                    for k, bs in enumerate(sets)]
    G.replay_ms(fixed_graphs, 2)
    fixed_ms = G.replay_ms(fixed_graphs, args.steps)
    del fixed_graphs, step_graphs

    # ------------------------------------------------ per-call times (cold)
    per_call = {}
    for name, (fn, bpp_unique, uses_x) in families.items():
        if name == "permute_copy_sorted":  # the stratified resampler's (sorted) ancestors
            for bs in sets:
                rs.resample_stratified(bs["lw"], 7, 0, anc=bs["anc"], ws=ws)
        touched = bpp_unique * P * n_sets + (8 * P * D * n_x if uses_x else 0)
        g = G.capture(lambda fn=fn: [fn(bs, k) for k, bs in enumerate(sets)])
        ms = [m / n_sets for m in G.replay_ms([g], 8)]
        del g
        per_call[name] = {"us": float(np.mean(ms)) * 1e3, "us_p50": pct(ms, 50) * 1e3,
                          "bytes_touched_per_replay": int(touched),
                          "cold": bool(touched > 2 * MALL_BYTES)}
        log(f"bench: {name} {per_call[name]['us']:.1f} us per call (cold)")
    for bs in sets:  # leave sorted ancestors behind
        rs.resample_stratified(bs["lw"], 7, 0, anc=bs["anc"], ws=ws)

    roofline = metropolis_roofline(torch, rs, G, sets[0]["lw"], per_call["metropolis"]["us"],
                                   P, B_eq5)
    roofline_hbm = hbm_summary(per_call, P, D)
    roofline_hbm["by_P"] = hbm_by_P(torch, rs, G, D, workloads)

    step_s = {"p50_ms": pct(step_ms, 50), "p99_ms": p99, "mean_ms": float(np.mean(step_ms))}
    full = {
        "metric": "resampled particles/s at P=2^20 (Metropolis B vs stratified) by weight var; p99",
        "value": value, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": float(np.mean(step_ms)),
        "p50_ms_per_step": pct(step_ms, 50), "p99_ms_per_step": p99,
        "wall_s_timed": wall, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 log-weights / f64 prefix sums / u32 Philox",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "P": P, "D": D, "sigma": sigma,
                   "metropolis_B": f"eq. (5), eps={EPS} (B={B_eq5} for buffer set 0)",
                   "buffer_sets": n_sets, "state_pairs": n_x, "parallelism": "single GPU"},
        "step": step_s,
        "step_fixed_B": {"B": args.B, "B_eq5": B_eq5, "converged": args.B >= B_eq5,
                         "p50_ms": pct(fixed_ms, 50), "p99_ms": pct(fixed_ms, 99),
                         "particles_per_s_p99": 4 * P / (pct(fixed_ms, 99) * 1e-3)},
        "per_call": per_call, "roofline": roofline, "roofline_hbm": roofline_hbm,
        "device": torch.cuda.get_device_name(0),
    }
    del sets
    torch.cuda.empty_cache()
    sections = []
    if not args.no_sweep:
        sections.append(("sweep", lambda: sweep(torch, rs, workloads, args)))
    if not args.no_batch:
        sections.append(("batched", lambda: batched(torch, rs, workloads, args)))
    sections.append(("minimal_copy", lambda: minimal_copy(torch, rs, workloads, P, B_eq5)))
    if not args.no_dirichlet:
        sections.append(("dirichlet", lambda: dirichlet(torch, rs, workloads, args)))
    if not args.no_filter:
        sections.append(("filter", lambda: filter_run(torch, workloads, args)))
        sections.append(("pmcmc", lambda: pmcmc_run(torch, workloads, args)))
    if args.serve_seconds > 0:
        sections.append(("serving", lambda: serving(torch, args)))
    if not args.no_cpu_baseline:
        sections.append(("cpu_baseline", lambda: cpu_baseline(torch, rs, args, workloads)))
    for name, fn in sections:
        t = time.perf_counter()
        full[name] = fn()
        log(f"bench: {name} done in {time.perf_counter() - t:.1f} s")
    full["bench_wall_s"] = time.perf_counter() - t_start
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        with open(args.out, "w") as f:
            json.dump(full, f)
            f.write("\n")
    print(json.dumps(headline(full, args.out)), flush=True)


WORKLOAD = ("resampler sweep point P=2^20, lw ~ N(0, 1), D=4 state copy; step = "
            "Metropolis (B from eq. (5), eps 0.01) + stratified + systematic + multinomial, "
            "each with the state copy (fused into the stratified/systematic fill, which "
            "writes ancestors, offspring and rows in one pass); cold HBM (rotating buffer sets)")


def call_families(rs, ws, B_eq5, B_fixed):
    """Per-call timing families: (call(bs, k), unique bytes per particle of
    one call's own buffers, whether it touches the state rows)."""
    def fused(kind):
        return lambda bs, k: rs.resample_and_copy(
            kind, bs["lw"], bs["x"], k, 0, B=B_eq5, anc=bs["anc"],
            off=bs["off"] if kind in ("stratified", "systematic") else None, x_out=bs["xo"],
            ws=None if kind == "metropolis" else ws)
    return {
        "metropolis": (lambda bs, k: rs.resample_metropolis(bs["lw"], B_eq5, k, 0, anc=bs["anc"]),
                       8, False),
        "metropolis_adaptive": (lambda bs, k: rs.resample_metropolis_adaptive(
            bs["lw"], k, 0, eps=EPS, B_max=B_MAX, anc=bs["anc"], ws=ws), 8, False),
        f"metropolis_B{B_fixed}": (lambda bs, k: rs.resample_metropolis(bs["lw"], B_fixed, k, 0,
                                                                       anc=bs["anc"]), 8, False),
        "stratified": (lambda bs, k: rs.resample_stratified(bs["lw"], k, 0, anc=bs["anc"], ws=ws,
                                                            off=bs["off"]), 12, False),
        "systematic": (lambda bs, k: rs.resample_systematic(bs["lw"], k, 0, anc=bs["anc"], ws=ws,
                                                            off=bs["off"]), 12, False),
        "multinomial": (lambda bs, k: rs.resample_multinomial(bs["lw"], k, 0, anc=bs["anc"],
                                                              ws=ws), 8, False),
        # the copy after the multinomial call (random ancestors), then after
        # stratified ancestors (sorted: the rows stream)
        "permute_copy_random": (lambda bs, k: rs.permute_copy(bs["anc"], bs["x"], x_out=bs["xo"]),
                                4, True),
        "permute_copy_sorted": (lambda bs, k: rs.permute_copy(bs["anc"], bs["x"], x_out=bs["xo"]),
                                4, True),
        "stratified_and_copy": (fused("stratified"), 12, True),
        "systematic_and_copy": (fused("systematic"), 12, True),
        "multinomial_and_copy": (fused("multinomial"), 8, True),
        "metropolis_and_copy": (fused("metropolis"), 8, True),
        # the one-launch form of the stratified resampler with the copy
        # (rs_prefix_set_path; the path is read when a call is enqueued)
        "stratified_and_copy_onepass": (lambda bs, k: (
            rs.rs_prefix_set_path("onepass"), fused("stratified")(bs, k),
            rs.rs_prefix_set_path("auto")), 12, True),
    }


def profile_only(torch, rs, args, sets, families, step):
    """Profiling mode: plain launches of one call family on the cold sets,
    with HIP events around the timed calls (back to back on one stream), so
    a profiler's per-kernel average can be set beside the same run's."""
    big = torch.empty(1 << 24, dtype=torch.float32, device=sets[0]["lw"].device)  # 64 MiB
    big_out = torch.empty_like(big)
    only = {name: fn for name, (fn, _, _) in families.items()}
    only["copycal"] = lambda bs, k: big_out.copy_(big)
    only["step"] = lambda bs, k: step(bs, k, 0)
    only["permute_copy"] = only["permute_copy_sorted"]
    probe_out = torch.empty(1 << 20, dtype=torch.float32, device=sets[0]["lw"].device)
    ip_ws = torch.empty(int(rs.lib.rs_inplace_workspace_bytes(sets[0]["lw"].numel())),
                        dtype=torch.uint8, device=sets[0]["lw"].device)
    only["inplace"] = lambda bs, k: rs.offspring_update_inplace(bs["off"], bs["x"], ws=ip_ws)
    only["gather_probe"] = lambda bs, k: rs.rs_probe_gather(sets[0]["lw"], 1 << 20, 8, k + 1,
                                                           out=probe_out)
    only["permute_copy_metropolis"] = only["permute_copy_random"]
    off_ws = torch.empty(int(rs.lib.rs_offspring_workspace_bytes(sets[0]["lw"].numel())),
                         dtype=torch.uint8, device=sets[0]["lw"].device)
    only["offspring"] = lambda bs, k: rs.ancestors_to_offspring(bs["anc"], off=bs["off"])
    only["offspring_ws"] = lambda bs, k: rs.ancestors_to_offspring_ws(bs["anc"], off=bs["off"],
                                                                      ws=off_ws)
    if args.only == "batched_metropolis":  # the batched configuration's Metropolis half
        from paper_1202_6163_amd import workloads
        from paper_1202_6163_amd.batch import Batch
        _, insts = batch_workload(torch, workloads, sets[0]["lw"].device)
        half = Batch([d for d in insts if d["kind"] == "metropolis"])
        only["batched_metropolis"] = lambda bs, k: half.run()
    fn = only[args.only]
    for k, bs in enumerate(sets):
        if args.only in ("inplace", "permute_copy_metropolis", "offspring", "offspring_ws"):
            # Metropolis ancestors (eq. (5)'s B) and their offspring
            families["metropolis"][0](bs, 900 + k)
            rs.ancestors_to_offspring(bs["anc"], off=bs["off"])
        else:  # sorted ancestors for the copy
            rs.resample_stratified(bs["lw"], 1, 0, anc=bs["anc"],
                                   ws=rs.workspace(bs["lw"].numel(), rs.MULTINOMIAL))
    for k in range(args.warmup):
        fn(sets[k % len(sets)], k)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(args.warmup, args.warmup + args.steps):
        fn(sets[k % len(sets)], k)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / max(args.steps, 1)
    print(f"profiled {args.only}: {args.warmup + args.steps} calls; {us:.2f} us per timed call "
          f"(HIP events, {args.steps} calls)", flush=True)


def metropolis_roofline(torch, rs, G, lw, us, P, B):
    """The dominant kernel, metropolis_kernel, against the L2 request rate:
    every iteration gathers one 4-byte proposed weight at a random index of
    the 4 MiB weight array, one L2 request each (the per-CU L1 holds under
    1 % of the array). Beside it the VALU view and the measured ceilings."""
    iters = float(P) * B
    rate = iters / (us * 1e-6)
    alu = iters * METRO_SLOTS_PER_ITER / (us * 1e-6) / 1e12
    meas = ceilings(torch, rs, G, lw, rate)
    return {"bound": "l2", "achieved": rate / 1e9, "peak": L2_PEAK_GREQ_S, "unit": "Greq/s",
            "frac": rate / 1e9 / L2_PEAK_GREQ_S, "traffic": load_traffic("metropolis"),
            "kernel": "metropolis_kernel", "avg_launch_us": us,
            "units_per_launch": {"chain_iterations": iters, "B": B, "P": P},
            "algorithmic_per_unit": {"l2_requests": 1, "gather_bytes": 4,
                                     "valu_slots": METRO_SLOTS_PER_ITER},
            "alu_view": {"achieved": alu, "peak": VALU_SLOTS_PER_S / 1e12,
                         "unit": "TVALU-slot/s", "frac": alu / (VALU_SLOTS_PER_S / 1e12)},
            "measured_ceilings": meas}


def hbm_summary(per_call, P, D):
    """The scan + state-copy path against HBM at P (cold per-call times)."""
    out = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s"}

    def entry(us, bpp, **kw):
        gbs = bpp * P / (us * 1e-6) / 1e9
        return dict(achieved=gbs, frac=gbs / HBM_PEAK_GBS, us=us, bytes_per_particle=bpp, **kw)
    out["permute_copy"] = entry(per_call["permute_copy_sorted"]["us"], 4 + 8 * D)
    out["stratified"] = entry(per_call["stratified"]["us"], 12,
                              outputs="ancestors and offspring")
    out["stratified_plus_copy"] = entry(per_call["stratified"]["us"] +
                                        per_call["permute_copy_sorted"]["us"], 12 + 4 + 8 * D,
                                        form="two calls")
    out["stratified_and_copy"] = entry(per_call["stratified_and_copy"]["us"], 12 + 4 + 8 * D,
                                       form="resample_and_copy (copy in the fill)")
    out["systematic_and_copy"] = entry(per_call["systematic_and_copy"]["us"], 12 + 4 + 8 * D,
                                       form="resample_and_copy (copy in the fill)")
    out["single_pass"] = entry(per_call["stratified_and_copy_onepass"]["us"], 12 + 4 + 8 * D,
                               form="stratified resample_and_copy in one launch (tile sums "
                                    "exchanged as tagged words; opt-in, slower)")
    out["note"] = ("bytes per particle as the method must move them: lw read twice, "
                   "ancestors written, (copy) ancestors read, rows read and written")
    return out


def headline(full, out_path):
    """The compact last stdout line (kept under 4 KB)."""
    r = full["roofline"]
    h = {k: full[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup",
                              "ms_per_step", "p50_ms_per_step", "p99_ms_per_step",
                              "higher_is_better", "scaling", "vs_baseline", "dtype", "data")}
    c = full["config"]
    h["config"] = {"workload": c["workload"], "P": c["P"], "D": c["D"], "sigma": c["sigma"],
                   "metropolis_B": c["metropolis_B"], "parallelism": c["parallelism"]}
    h["roofline"] = {k: r[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                       "kernel", "avg_launch_us")}
    h["roofline"]["alu_frac"] = r["alu_view"]["frac"]
    mc = r["measured_ceilings"]
    h["roofline"]["measured"] = {"gather_per_s": mc["random_gather_per_s"],
                                 "frac_of_gather_probe": mc["frac_of_measured_ceiling"]}
    hb = full["roofline_hbm"]
    h["roofline_hbm"] = {k: {"frac": hb[k]["frac"], "us": hb[k]["us"]}
                         for k in ("permute_copy", "stratified", "stratified_plus_copy",
                                   "stratified_and_copy", "systematic_and_copy") if k in hb}
    if "single_pass" in hb:
        h["roofline_hbm"]["single_pass"] = {"frac": hb["single_pass"]["frac"],
                                            "us": hb["single_pass"]["us"]}
    h["per_call_us"] = {k: round(v["us"], 2) for k, v in full["per_call"].items()}
    h["step_fixed_B"] = {k: full["step_fixed_B"][k] for k in ("B", "B_eq5", "converged",
                                                               "p99_ms")}
    if "sweep" in full:
        h["crossover_sigma_by_P"] = full["sweep"]["crossover_sigma_by_P"]
    if "batched" in full:
        b = full["batched"]
        h["batched"] = {"ms_p50": b["batched_ms_p50"],
                        "speedup_vs_per_instance_graph": b["speedup_vs_per_instance_graph"]}
    if "minimal_copy" in full:
        h["minimal_copy"] = {k: {m: v[m] for m in ("permute_copy_us", "inplace_us",
                                                     "anc_to_off_plus_inplace_us",
                                                     "anc_to_off_ws_plus_inplace_us",
                                                     "bytes_ratio_vs_permute_copy")}
                             for k, v in full["minimal_copy"].items() if k.startswith("D")}
    if "serving" in full:
        h["serving"] = {name: {k: pt.get(k) for k in ("rate_req_per_s", "p50_latency_ms",
                                                      "p99_latency_ms", "particles_per_s",
                                                      "mean_batch")}
                        for name, pt in full["serving"].items() if isinstance(pt, dict)}
    if "cpu_baseline" in full:
        cb = full["cpu_baseline"]
        h["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        h["cpu_baseline"]["all_cores"] = {k: cb["all_cores"][k]
                                          for k in ("value", "cores")}
        h["parity"] = cb["parity"]
    h["full_results"] = out_path
    h = _round_floats(h)
    line = json.dumps(h)
    for drop in ("per_call_us", "crossover_sigma_by_P", "serving", "batched"):
        if len(line) <= 4000:
            break
        h.pop(drop, None)
        line = json.dumps(h)
    return h


def _round_floats(v, sig=5):
    """Floats to `sig` significant digits, recursively (keeps the line short)."""
    if isinstance(v, float):
        return float(f"{v:.{sig}g}") if math.isfinite(v) else v
    if isinstance(v, dict):
        return {k: _round_floats(x, sig) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_round_floats(x, sig) for x in v]
    return v


def ceilings(torch, rs, G, lw, metro_iter_per_s):
    """Measured device rates for the two halves of a Metropolis iteration:
    random 4-byte gathers from the P weights (the proposal) and Philox4x32-10
    blocks (two words per iteration). The iteration rate can exceed neither
    the gather rate nor twice the block rate."""
    threads, rounds = 1 << 20, 8
    out_f = torch.empty(threads, dtype=torch.float32, device=lw.device)
    out_i = torch.empty(threads, dtype=torch.int32, device=lw.device)
    g1 = G.capture(lambda: rs.rs_probe_gather(lw, threads, rounds, 1, out=out_f))
    g2 = G.capture(lambda: rs.rs_probe_philox(threads, rounds, 1, out=out_i))
    G.replay_ms([g1, g2], 2)
    gather_ms = float(np.median(G.replay_ms([g1], 10)))
    philox_ms = float(np.median(G.replay_ms([g2], 10)))
    gathers = threads * rounds * 8 / (gather_ms * 1e-3)
    blocks = threads * rounds * 4 / (philox_ms * 1e-3)
    bound = min(gathers, 2 * blocks)
    # the gather rate against the size of the gathered array (L2 is 4 MB per XCD)
    by_size = {}
    for lg in (16, 18, 19, 20, 21, 22, 24):
        arr = torch.zeros(1 << lg, dtype=torch.float32, device=lw.device)
        g = G.capture(lambda arr=arr: rs.rs_probe_gather(arr, threads, rounds, 1, out=out_f))
        G.replay_ms([g], 2)
        ms = float(np.median(G.replay_ms([g], 6)))
        by_size[str(4 << lg)] = threads * rounds * 8 / (ms * 1e-3)
    return {"random_gather_per_s": gathers, "philox_blocks_per_s": blocks,
            "metropolis_iter_per_s": metro_iter_per_s, "iteration_ceiling_per_s": bound,
            "frac_of_measured_ceiling": metro_iter_per_s / bound,
            "gather_array_bytes": 4 * lw.numel(), "random_gather_per_s_by_array_bytes": by_size}


def hbm_by_P(torch, rs, G, D, workloads):
    """Stratified (ancestors + offspring), with the state copy as its own
    launch and fused into the fill, against HBM at growing P (cold: enough
    rotating buffer sets that each graph touches COLD_BYTES of its own
    buffers): the fixed latency of the dependent launches is amortised as P
    grows."""
    dev = torch.device("cuda", 0)
    res = {}
    for lg in (22, 24):
        P = 1 << lg
        ns = max(2, -(-COLD_BYTES // (12 * P)))
        nx = max(2, -(-COLD_BYTES // (8 * P * D)))
        xs = [(torch.randn(P, D, device=dev), torch.empty(P, D, device=dev)) for _ in range(nx)]
        sets = [dict(lw=torch.randn(P, device=dev), anc=torch.empty(P, dtype=torch.int32, device=dev),
                     off=torch.empty(P, dtype=torch.int32, device=dev)) for _ in range(ns)]
        ws = rs.workspace(P, rs.MULTINOMIAL, dev)

        def body(form):
            for k, bs in enumerate(sets):
                x, xo = xs[k % nx]
                if form == "fused":
                    rs.resample_and_copy("stratified", bs["lw"], x, k, 0, anc=bs["anc"],
                                         off=bs["off"], x_out=xo, ws=ws)
                    continue
                rs.resample_stratified(bs["lw"], k, 0, anc=bs["anc"], ws=ws, off=bs["off"])
                if form == "copy":
                    rs.permute_copy(bs["anc"], x, x_out=xo)
        entry = {"buffer_sets": ns, "state_pairs": nx}
        for name, form, bpp in (("stratified", "plain", 12),
                                ("stratified_plus_copy", "copy", 12 + 4 + 8 * D),
                                ("stratified_and_copy", "fused", 12 + 4 + 8 * D)):
            g = G.capture(lambda form=form: body(form))
            G.replay_ms([g], 2)
            us = float(np.median(G.replay_ms([g], 6))) * 1e3 / ns
            del g
            gbs = bpp * P / (us * 1e-6) / 1e9
            entry[name] = {"us": us, "achieved": gbs, "frac": gbs / HBM_PEAK_GBS,
                           "bytes_per_particle": bpp}
        res[f"2^{lg}"] = entry
        del sets, xs
        torch.cuda.empty_cache()
    return res


def load_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current sources of that kernel family (null otherwise)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    entry = rec.get(kernel)
    if not entry or entry.get("source_sha256") != source_hash(kernel):
        return None
    return entry.get("bytes_per_launch")


# Kernels of each call family, by a part of their names (the --only runs also
# launch set-up stratified calls, whose table and fill kernels are left out
# of the other families).
FAMILY_KERNELS = {
    "copycal": ["copyBuffer"],
    "metropolis": ["metropolis_kernel"],
    "permute_copy": ["copy_rows"],
    "stratified": ["tile_reduce_kernel", "table_kernel<0", "fill_kernel<0"],
    "multinomial": ["tile_reduce_kernel", "cumulative_kernel", "multinomial_search_kernel"],
    "inplace": ["ip_count_kernel", "ip_table_kernel", "ip_move_kernel"],
    "permute_copy_metropolis": ["copy_rows"],
}
CALIBRATION_BYTES = 64 << 20  # the copycal run copies 64 MiB per dispatch


def record_traffic(pmc_dir):
    """profiles/traffic.json from rocprofv3 --pmc runs of `bench.py --only X`
    (one counter per run, directories <family>_<COUNTER>): per kernel the
    counter's mean per dispatch, scaled by what the same counter reads for a
    plain 64 MiB copy, and per family the sum over its kernels."""
    import csv
    import glob

    def per_dispatch(family, counter):
        files = glob.glob(os.path.join(pmc_dir, f"{family}_{counter}", "**",
                                       "*counter_collection.csv"), recursive=True)
        vals = {}
        for path in files:
            with open(path, newline="") as f:
                for row in csv.DictReader(f):
                    if row.get("Counter_Name") != counter:
                        continue
                    name = row["Kernel_Name"]
                    if any(k in name for k in FAMILY_KERNELS[family]):
                        vals.setdefault(name, {}).setdefault(row.get("Dispatch_Id"), 0.0)
                        vals[name][row.get("Dispatch_Id")] += float(row["Counter_Value"])
        return {name: float(np.mean(list(d.values()))) for name, d in vals.items()}

    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:  # families not measured in this directory keep their entries
        rec = json.load(open(path))
    except (OSError, ValueError):
        rec = {}
    factor = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        cal = per_dispatch("copycal", counter)
        if cal:
            kib = float(np.mean(list(cal.values())))
            rec.setdefault("_calibration", {})[counter] = {
                "factor": CALIBRATION_BYTES / (kib * 1024.0), "kernel": "copyBuffer (torch)",
                "KiB_per_dispatch": kib}
        factor[counter] = rec["_calibration"][counter]["factor"]
    for family in ("metropolis", "permute_copy", "stratified", "multinomial", "inplace",
                   "permute_copy_metropolis"):
        kernels = {}
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            for name, kib in per_dispatch(family, counter).items():
                kernels.setdefault(name[:80], {})[counter] = kib * 1024.0 * factor[counter]
        if not kernels:
            continue
        total = sum(sum(v.values()) for v in kernels.values())
        rec[family] = {"bytes_per_launch": total, "kernels": kernels,
                       "source_sha256": source_hash(family),
                       "bench_args": "--D 16" if family in ("inplace", "permute_copy_metropolis")
                       else "--D 4"}
        log(f"traffic: {family} {total / 1e6:.2f} MB per call")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


# The sources each kernel family is compiled from (what invalidates its counters).
KERNEL_SOURCES = {
    "metropolis": ["metropolis.hip", "metropolis_impl.h", "common.h", "launch.h"],
    "permute_copy": ["misc.hip", "common.h", "launch.h"],
    "stratified": ["prefix.hip", "prefix_impl.h", "prefix.h", "analysis.h", "common.h", "launch.h"],
    "multinomial": ["prefix.hip", "prefix_impl.h", "prefix.h", "analysis.h", "common.h", "launch.h"],
    "inplace": ["inplace.hip", "prefix.h", "common.h", "launch.h"],
    "permute_copy_metropolis": ["misc.hip", "common.h", "launch.h"],
}


def _code_only(text):
    """C++ source without its comments and blank lines (a comment edit does
    not change the kernel the counters measured)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def source_hash(kernel):
    """Hash of the kernel family's code (comments stripped), plus the stored
    launch tuning for Metropolis (it selects the kernel variant that runs)."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_1202_6163_amd")
    files = [os.path.join("csrc", name) for name in sorted(KERNEL_SOURCES[kernel])]
    if kernel == "metropolis":
        files.append("tuning.json")
    for name in files:
        try:
            with open(os.path.join(pkg, name), "r", encoding="utf-8") as f:
                text = f.read()
            if name.endswith((".hip", ".h", ".cpp")):
                text = _code_only(text)
            h.update(name.encode() + text.encode())
        except OSError:
            h.update(name.encode() + b"<missing>")
    return h.hexdigest()


def sweep(torch, rs, workloads, args):
    """Warm-cache p50/p99 particles/s per (P, sigma, resampler[, B]), accuracy
    metric, ESS, eq. (5) B and the Metropolis-vs-stratified crossover."""
    dev = torch.device("cuda", 0)
    G = Graphs(torch)
    res = {"note": "warm cache (buffers reused); per-call time = a graph replay of R "
                   "back-to-back calls / R; p50/p99 over replays", "points": []}
    Ps = [1 << int(v) for v in args.sweep_P.split(",") if v]
    D = args.D
    for P in Ps:
        ws = rs.workspace(P, rs.MULTINOMIAL, dev)
        x = torch.from_numpy(workloads.state_rows_normal(P, D, 0)).to(dev)
        xo = torch.empty_like(x)
        anc = torch.empty(P, dtype=torch.int32, device=dev)
        off = torch.empty(P, dtype=torch.int32, device=dev)
        for sigma in workloads.SIGMAS:
            lw = torch.from_numpy(workloads.normal_logweights(P, sigma, 0)).to(dev)
            w = torch.exp(lw.double() - lw.max().double())
            W = w.sum()
            p = (w / W)
            ess = float(1.0 / (p * p).sum())
            wmax = float(p.max())
            point = {"P": P, "sigma": sigma, "ess_frac": ess / P,
                     "B_eq5_eps1e-2": rs.metropolis_B(P, wmax, 1e-2),
                     "B_eq5_eps1e-3": rs.metropolis_B(P, wmax, 1e-3), "resamplers": {}}

            def measure(call, with_copy, r_min=1):
                # calls per graph: about 2e5 particles of work, and at least
                # r_min (4 for the short prefix calls, so a replay's own launch
                # cost is spread over several calls at every P)
                R = max(r_min, min(64, int(2e5 // P) + 1))

                def body():
                    for k in range(R):
                        call(k)
                        if with_copy:
                            rs.permute_copy(anc, x, x_out=xo)
                g = G.capture(body)
                ms = [m / R for m in G.replay_ms([g], args.reps)]
                return {"p50_pps": P / (pct(ms, 50) * 1e-3), "p99_pps": P / (pct(ms, 99) * 1e-3),
                        "p50_us": pct(ms, 50) * 1e3, "p99_us": pct(ms, 99) * 1e3,
                        "calls_per_graph": R}

            def accuracy(call):
                errs = []
                for s in range(4):
                    call(100 + s)
                    rs.ancestors_to_offspring(anc, off=off)
                    e = ((off.double() / P - p) ** 2).sum()
                    errs.append(float(e))
                return float(np.mean(errs))

            calls = {"stratified": lambda k: rs.resample_stratified(lw, k, 0, anc=anc, ws=ws),
                     "systematic": lambda k: rs.resample_systematic(lw, k, 0, anc=anc, ws=ws),
                     "multinomial": lambda k: rs.resample_multinomial(lw, k, 0, anc=anc, ws=ws)}
            for Bm in workloads.SWEEP_B:
                calls[f"metropolis_B{Bm}"] = (
                    lambda k, Bm=Bm: rs.resample_metropolis(lw, Bm, k, 0, anc=anc))
            for name, call in calls.items():
                r_min = 1 if name.startswith("metropolis") else 4
                r = measure(call, False, r_min)
                r["with_copy"] = measure(call, True, r_min)
                r["error"] = accuracy(call)
                point["resamplers"][name] = r
            strat = point["resamplers"]["stratified"]["p99_pps"]
            faster = [Bm for Bm in workloads.SWEEP_B
                      if point["resamplers"][f"metropolis_B{Bm}"]["p99_pps"] > strat]
            point["metropolis_faster_up_to_B"] = max(faster) if faster else 0
            need = point["B_eq5_eps1e-2"]
            point["metropolis_converged_faster"] = bool(faster) and need <= max(faster)
            res["points"].append(point)
            print(f"sweep P={P} sigma={sigma}: stratified {strat:.3e} p/s, Metropolis faster up "
                  f"to B={point['metropolis_faster_up_to_B']}, eq5 B={need}", file=sys.stderr,
                  flush=True)
    cross = {}
    for P in Ps:
        pts = [q for q in res["points"] if q["P"] == P]
        wins = [q["sigma"] for q in pts if q["metropolis_converged_faster"]]
        cross[str(P)] = max(wins) if wins else None
    res["crossover_sigma_by_P"] = cross
    res["crossover_note"] = ("largest swept sigma at which Metropolis with the eq. (5) B "
                             "(eps = 0.01, rounded up to the swept B grid) is faster than "
                             "stratified at p99; null: never")
    return res


def dirichlet(torch, rs, workloads, args):
    """Sec. 3's own experiment: Dirichlet(alpha) weights, P = 256 .. 65536,
    alpha in {10, 1, .1, .01}; accuracy metric sum (o/P - w/W)^2 averaged over
    R resamplings and per-call time for multinomial, stratified, systematic,
    Metropolis at eq. (5)'s B (eps = 0.01, capped at 4096) and the
    sorted-weight multinomial and systematic. Per-call times: eager calls
    (events around R back-to-back calls, host dispatch included) and the GPU
    time of a graph of R calls, for every resampler."""
    dev = torch.device("cuda", 0)
    R = args.dirichlet_R
    G = Graphs(torch)
    out = {"note": "us_per_call: eager per-call time (host dispatch included); "
                   "us_per_call_graph: GPU time per call in a graph of R calls; error averaged "
                   "over R resamplings with different seeds",
           "R": R, "points": []}
    for P in (256, 1024, 4096, 16384, 65536):
        anc = torch.empty(P, dtype=torch.int32, device=dev)
        off = torch.empty(P, dtype=torch.int32, device=dev)
        ws = rs.workspace(P, rs.MULTINOMIAL, dev)
        ws_sorted = torch.empty(max(rs.lib.rs_sorted_workspace_bytes(P, rs.MULTINOMIAL),
                                    rs.lib.rs_sorted_workspace_bytes(P, rs.SYSTEMATIC)),
                                dtype=torch.uint8, device=dev)
        for alpha in (10.0, 1.0, 0.1, 0.01):
            lw_h = workloads.dirichlet_logweights(P, alpha, 7)
            lw = torch.from_numpy(lw_h).to(dev)
            p = torch.exp(lw.double() - lw.max().double())
            p = p / p.sum()
            B = min(rs.metropolis_B(P, float(p.max()), 1e-2), 4096)
            calls = {
                "multinomial": lambda k: rs.resample_multinomial(lw, k, 0, anc=anc, ws=ws),
                "stratified": lambda k: rs.resample_stratified(lw, k, 0, anc=anc, ws=ws),
                "systematic": lambda k: rs.resample_systematic(lw, k, 0, anc=anc, ws=ws),
                "metropolis_eq5": lambda k: rs.resample_metropolis(lw, B, k, 0, anc=anc),
                "multinomial_sorted": lambda k: rs.resample_sorted("multinomial", lw, k, 0,
                                                                   anc=anc, ws=ws_sorted),
                "systematic_sorted": lambda k: rs.resample_sorted("systematic", lw, k, 0,
                                                                  anc=anc, ws=ws_sorted),
            }
            point = {"P": P, "alpha": alpha, "ess_frac": float(1.0 / (p * p).sum()) / P,
                     "B_eq5": B, "resamplers": {}}
            for name, call in calls.items():
                errs = []
                for k in range(R):
                    call(500 + k)
                    rs.ancestors_to_offspring(anc, off=off)
                    errs.append(((off.double() / P - p) ** 2).sum())
                err = float(torch.stack(errs).mean())
                for k in range(3):
                    call(k)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for k in range(R):
                    call(900 + k)
                e1.record()
                torch.cuda.synchronize()
                point["resamplers"][name] = {"error": err, "us_per_call": e0.elapsed_time(e1) * 1e3 / R}
                g = G.capture(lambda call=call: [call(900 + k) for k in range(R)])
                ms = G.replay_ms([g], 3)
                point["resamplers"][name]["us_per_call_graph"] = pct(ms, 50) * 1e3 / R
            out["points"].append(point)
            print(f"dirichlet P={P} alpha={alpha}: " + ", ".join(
                f"{k} {v['us_per_call']:.1f}us ({v.get('us_per_call_graph', float('nan')):.1f} in a graph)"
                for k, v in point["resamplers"].items()),
                file=sys.stderr, flush=True)
    return out


def minimal_copy(torch, rs, workloads, P, B):
    """The state update after Metropolis (random ancestors, eq. (5)'s B) at P,
    D = 4 and 16, cold: the ancestor-indexed copy into a second buffer
    against the in-place minimal-copy update (offspring form), with and
    without the ancestors-to-offspring conversion (atomic form, and the
    workspace form with one reused workspace). Algorithmic HBM bytes per
    particle: copy 4 + 8D; in place 8D per hole + 8 (the counts read twice)
    + 4 (a source tile's counts), the conversion 12 (ancestors read, counts
    cleared and counted)."""
    dev = torch.device("cuda", 0)
    G = Graphs(torch)
    res = {"note": "Metropolis ancestors at eq. (5)'s B; cold buffer sets (> 512 MiB per "
                   "graph); per-call mean of graph replays"}
    for D in (4, 16):
        n_sets = max(4, -(-COLD_BYTES // (P * (8 * D + 12))))
        sets = []
        for k in range(n_sets):
            lw = torch.from_numpy(workloads.normal_logweights(P, 1.0, 500 + k)).to(dev)
            anc = rs.resample_metropolis(lw, B, 700 + k, 0)
            off = rs.ancestors_to_offspring(anc)
            x = torch.from_numpy(workloads.state_rows_normal(P, D, k)).to(dev)
            sets.append({"anc": anc, "off": off, "off2": torch.empty_like(off), "x": x,
                         "xo": torch.empty_like(x),
                         "ws": torch.empty(int(rs.lib.rs_inplace_workspace_bytes(P)),
                                           dtype=torch.uint8, device=dev)})
            del lw
        holes = float(np.mean([(bs["off"] == 0).float().mean().item() for bs in sets]))
        off_ws = torch.empty(int(rs.lib.rs_offspring_workspace_bytes(P)), dtype=torch.uint8,
                             device=dev)
        forms = {
            "permute_copy_us": lambda bs: rs.permute_copy(bs["anc"], bs["x"], x_out=bs["xo"]),
            "inplace_us": lambda bs: rs.offspring_update_inplace(bs["off"], bs["x"], ws=bs["ws"]),
            "anc_to_off_us": lambda bs: rs.ancestors_to_offspring(bs["anc"], off=bs["off2"]),
            "anc_to_off_ws_us": lambda bs: rs.ancestors_to_offspring_ws(bs["anc"], off=bs["off2"],
                                                                        ws=off_ws),
            "anc_to_off_plus_inplace_us": lambda bs: (
                rs.ancestors_to_offspring(bs["anc"], off=bs["off2"]),
                rs.offspring_update_inplace(bs["off2"], bs["x"], ws=bs["ws"])),
            "anc_to_off_ws_plus_inplace_us": lambda bs: (
                rs.ancestors_to_offspring_ws(bs["anc"], off=bs["off2"], ws=off_ws),
                rs.offspring_update_inplace(bs["off2"], bs["x"], ws=bs["ws"])),
        }
        out = {"holes_fraction": holes, "buffer_sets": n_sets}
        for name, fn in forms.items():
            g = G.capture(lambda fn=fn: [fn(bs) for bs in sets])
            G.replay_ms([g], 2)
            ms = G.replay_ms([g], 6)
            out[name] = float(np.mean(ms)) / n_sets * 1e3
            del g
        alg_copy = 4 + 8 * D
        alg_inplace = 8 * D * holes + 12
        out["bytes_per_particle"] = {"permute_copy": alg_copy, "inplace": alg_inplace,
                                     "anc_to_off_plus_inplace": alg_inplace + 12}
        out["bytes_ratio_vs_permute_copy"] = alg_inplace / alg_copy
        res[f"D{D}"] = out
        log(f"minimal_copy D={D}: holes {holes:.3f}; copy {out['permute_copy_us']:.1f} us, "
            f"in place {out['inplace_us']:.1f} us, with conversion "
            f"{out['anc_to_off_plus_inplace_us']:.1f} us (workspace form "
            f"{out['anc_to_off_ws_plus_inplace_us']:.1f} us)")
        del sets, off_ws
        torch.cuda.empty_cache()
    return res


def batch_workload(torch, workloads, dev):
    """The batched configuration's 1024 instances (sizes, then the instance
    dicts): P log-uniform in [2^8, 2^16], sigma in [0.25, 3], Metropolis B = 64
    and stratified alternating, D = 16 rows."""
    P, sig = workloads.batch_instances(1024, seed=0)
    insts = []
    for k in range(len(P)):
        Pk = int(P[k])
        insts.append(dict(
            lw=torch.from_numpy(workloads.normal_logweights(Pk, sig[k], k)).to(dev),
            anc=torch.empty(Pk, dtype=torch.int32, device=dev),
            kind="metropolis" if k % 2 else "stratified", B=64, seed=5, instance=k,
            x_in=torch.from_numpy(workloads.state_rows_normal(Pk, 16, k)).to(dev),
            x_out=torch.empty((Pk, 16), dtype=torch.float32, device=dev)))
    return P, insts


def batched(torch, rs, workloads, args):
    """1024 instances, P log-uniform in [2^8, 2^16], sigma in [0.25, 3],
    Metropolis B = 64 and stratified alternating, D = 16: one batched graph
    replay against the same work as per-instance calls (resample +
    permute_copy) captured in one graph, and launched one by one."""
    from paper_1202_6163_amd.batch import Batch
    dev = torch.device("cuda", 0)
    P, insts = batch_workload(torch, workloads, dev)
    total = int(P.sum())
    G = Graphs(torch)
    b = Batch(insts)
    gb = G.capture(b.run)
    ms_b = G.replay_ms([gb], 10)
    ws = rs.workspace(1 << 16, rs.STRATIFIED, dev)

    def per_instance():
        for d in insts:
            if d["kind"] == "metropolis":
                rs.resample_metropolis(d["lw"], d["B"], d["seed"], d["instance"], anc=d["anc"])
            else:
                rs.resample_stratified(d["lw"], d["seed"], d["instance"], anc=d["anc"], ws=ws)
            rs.permute_copy(d["anc"], d["x_in"], x_out=d["x_out"])
    gp = G.capture(per_instance)
    ms_p = G.replay_ms([gp], 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_instance()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3
    tb, tp = pct(ms_b, 50), pct(ms_p, 50)
    # the two halves on their own: the Metropolis instances' iterations per
    # second set beside the L2 request peak (an instance whose weights fit a
    # CU's 32 KB L1 is served partly there, so the ratio is not a roofline
    # fraction and may exceed 1; the counters of the profiling family
    # batched_metropolis give the L2 requests), the stratified ones against
    # HBM (lw twice, ancestors, the D = 16 copy: 12 + 4 + 128 B)
    halves = {}
    for kind in ("metropolis", "stratified"):
        sub = [d for d in insts if d["kind"] == kind]
        bk = Batch(sub)
        gk = G.capture(bk.run)
        msk = pct(G.replay_ms([gk], 10), 50)
        n_k = sum(int(d["lw"].numel()) for d in sub)
        h = {"instances": len(sub), "particles": n_k, "ms_p50": msk}
        if kind == "metropolis":
            it = n_k * 64
            l1_sized = sum(int(d["lw"].numel()) for d in sub if 4 * d["lw"].numel() <= L1_BYTES)
            h.update(iterations=it, iterations_per_s=it / (msk * 1e-3),
                     iterations_over_l2_request_peak=it / (msk * 1e-3) / (L2_PEAK_GREQ_S * 1e9),
                     iteration_share_in_l1_sized_instances=l1_sized / n_k)
        else:
            by = n_k * (12 + 4 + 8 * 16)
            h.update(bytes=by, GB_per_s=by / (msk * 1e-3) / 1e9,
                     frac_of_hbm_peak=by / (msk * 1e-3) / 1e9 / HBM_PEAK_GBS)
        halves[kind] = h
        del gk, bk
    return {"instances": len(P), "particles": total, "D": 16,
            "halves": halves,
            "batched_ms_p50": tb, "batched_ms_p99": pct(ms_b, 99),
            "per_instance_graph_ms_p50": tp, "per_instance_eager_ms": eager_ms,
            "batched_instances_per_s": len(P) / (tb * 1e-3),
            "batched_particles_per_s": total / (tb * 1e-3),
            "per_instance_graph_particles_per_s": total / (tp * 1e-3),
            "speedup_vs_per_instance_graph": tp / tb, "speedup_vs_eager": eager_ms / tb,
            "tuning": dict(chains_per_item=b.tuning.chains_per_item, unroll=b.tuning.unroll,
                           lds_max_p=b.tuning.lds_max_p, blocks=b.plan.blocks)}


def filter_run(torch, workloads, args):
    """Bootstrap filter, D = 8, T = 200, P = 2^18, resampling every step
    (stratified; Metropolis with B from eq. (5) per step), one HIP graph per
    run; log-likelihood against the Kalman filter."""
    from oracle.kalman import kalman_loglik
    from paper_1202_6163_amd.filter import BootstrapFilter
    A = workloads.filter_model(D=8, seed=0)
    y = workloads.filter_observations(A, T=200, seed=0)
    ll_true = kalman_loglik(A, y, 0.1, 0.5)
    res = {"P": 1 << 18, "D": 8, "T": 200, "kalman_loglik": ll_true}
    for resampler in ("stratified", "metropolis_adaptive"):
        f = BootstrapFilter(A, 1 << 18, seed=1, resampler=resampler, B=16384)
        yd = torch.as_tensor(y, device="cuda")
        lse = torch.empty(200, dtype=torch.float64, device="cuda")
        g = f.capture(yd, lse)
        G = Graphs(torch)
        ms = G.replay_ms([g], 5)
        res[resampler] = {"ms_per_run_p50": pct(ms, 50), "us_per_step": pct(ms, 50) * 1e3 / 200,
                          "loglik": f.loglik(lse)}
    return res


def pmcmc_run(torch, workloads, args):
    """Particle marginal Metropolis-Hastings over log q (Sec. 1's use of the
    filter): K = 64 chains, each iteration K filters of P = 4096 particles,
    D = 4, T = 100, run as one batch per time step; time per iteration
    against K single-filter runs of the same size, and the posterior summary
    against the Kalman grid posterior."""
    import math
    from oracle.kalman import kalman_loglik
    from paper_1202_6163_amd.filter import BootstrapFilter
    from paper_1202_6163_amd.pmcmc import BatchedFilters, pmmh
    K, P, T = 64, 4096, 100
    A = workloads.filter_model(D=4, seed=1)
    y = workloads.filter_observations(A, T=T, q=0.1, r=0.5, seed=3)
    yd = torch.from_numpy(y).cuda()
    bf = BatchedFilters(A, K, P, r=0.5, seed=11)
    bf.loglik(np.full(K, 0.1), yd, run=0)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_eval = 5
    for it in range(n_eval):
        bf.loglik(np.full(K, 0.1), yd, run=1 + it)
    batched_s = (time.perf_counter() - t0) / n_eval
    single = BootstrapFilter(A, P, q=0.1, r=0.5, seed=11)
    single.run(y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(8):
        single.run(y)
    single_s = (time.perf_counter() - t0) / 8 * K
    grid = np.linspace(math.log(0.01), math.log(1.0), 241)
    lp = np.array([kalman_loglik(A, y, math.exp(g), 0.5) for g in grid])
    lp += -0.5 * ((grid - math.log(0.1)) / 1.0) ** 2
    w = np.exp(lp - lp.max())
    w /= w.sum()
    pm = float((w * grid).sum())
    psd = float(math.sqrt((w * (grid - pm) ** 2).sum()))
    t0 = time.perf_counter()
    iters = 60
    chain, rate = pmmh(bf, yd, iters=iters, theta0=math.log(0.1), step=1.2 * psd, seed=4)
    pmmh_s = time.perf_counter() - t0
    samples = chain[20:].ravel()
    return {"K": K, "P": P, "T": T, "D": 4,
            "batched_s_per_iteration": batched_s, "single_filters_s_per_iteration": single_s,
            "speedup": single_s / batched_s,
            "filter_steps_per_s": K * T / batched_s,
            "particle_steps_per_s": K * T * P / batched_s,
            "pmmh_iterations": iters, "pmmh_seconds": pmmh_s, "acceptance": rate,
            "posterior_mean_log_q": float(samples.mean()), "posterior_sd_log_q": float(samples.std()),
            "grid_posterior_mean_log_q": pm, "grid_posterior_sd_log_q": psd,
            "note": "eager launches (5 per time step for all K filters); single = "
                    "BootstrapFilter.run per filter, eager"}


def serving(torch, args):
    """Poisson arrivals, P log-uniform, sigma from the client payload slots
    (uniform in [0.5, 4]), D in {1, 16}; Metropolis (eq. (5)'s B, capped at
    1024) for the low-variance slots, stratified or systematic for the rest;
    weights and state uploaded from pinned host memory
    at admission, admitted by footprint, continuously batched on 4 streams.
    Load points: the configured 2000 req/s with P in [2^10, 2^20]; then
    smaller requests (P in [2^10, 2^14]) at 8000 and 16000 req/s, where
    batches of many requests form, each also with every request in its own
    launches (max_batch = 1): at 8000 req/s both keep up and the latencies
    compare; at 16000 req/s the offered particles/s exceed what per-request
    launches sustain."""
    from paper_1202_6163_amd.serve import GpuExecutor, Payloads, make_requests, serve, summarize
    pay = Payloads(1 << 20)
    heavy_s = min(3.0, args.serve_seconds)
    points = (("config_load", 2000.0, args.serve_seconds, 20, 32 << 30, 256),
              ("small_8k", 8000.0, heavy_s, 14, 1 << 30, 256),
              ("small_8k_per_request_launches", 8000.0, heavy_s, 14, 1 << 30, 1),
              ("small_16k", 16000.0, heavy_s, 14, 1 << 30, 256),
              ("small_16k_per_request_launches", 16000.0, heavy_s, 14, 1 << 30, 1))
    out = {"note": "latency = server-observed completion - arrival on one host clock; "
                   "includes the host-to-device upload of weights and state"}
    for name, rate, secs, p_hi, budget, max_batch in points:
        reqs = make_requests(rate=rate, duration=secs, seed=0, p_hi=p_hi, B=1024)
        ex = GpuExecutor(n_streams=4, payloads=pay)
        sched = serve(reqs, ex, budget_bytes=budget, max_batch=max_batch)
        summ = summarize(sched, secs)
        summ.update({"rate_req_per_s": rate, "seconds": secs, "P_range": [1 << 10, 1 << p_hi],
                     "budget_bytes": budget, "streams": 4, "max_batch": max_batch,
                     "metropolis_B_cap": 1024})
        summ["p50_ms"], summ["p99_ms"] = summ["p50_latency_ms"], summ["p99_latency_ms"]
        out[name] = summ
        log(f"serving {name}: p50 {summ['p50_latency_ms']:.2f} ms p99 "
            f"{summ['p99_latency_ms']:.2f} ms, mean batch {summ['mean_batch']:.2f}, "
            f"{summ['particles_per_s']:.3e} particles/s")
        del ex, sched
    return out


def cpu_baseline(torch, rs, args, workloads):
    """The oracle (plain C, as committed) on a bounded sample of the step at
    P = 2^20: the stratified, systematic and multinomial resamplers in full,
    Metropolis with the step's eq. (5) B on every 16th chain (a chain's cost
    does not depend on which particle it starts from), offspring and the
    copies; single-threaded on one pinned core, and the OpenMP build of the
    same source on every core (Metropolis chains and copies in full). The
    GPU's outputs for the same inputs are compared with the oracle's: the
    Metropolis ancestors bit for bit, the others up to draws within 1e-6 of a
    boundary (counted), the copied rows bit for bit where the ancestors agree."""
    import oracle
    from tests.parity import count_mismatches
    P, D = args.P, args.D
    lw = workloads.normal_logweights(P, args.sigma, 0)
    x = workloads.state_rows_normal(P, D, 0)
    dev = torch.device("cuda", 0)
    lw_d, x_d = torch.from_numpy(lw).to(dev), torch.from_numpy(x).to(dev)
    ws = rs.workspace(P, rs.MULTINOMIAL, dev)
    Bd = torch.zeros(1, dtype=torch.int32, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    gpu = {"metropolis": rs.resample_metropolis_adaptive(lw_d, 1, 0, eps=EPS, B_max=B_MAX,
                                                         B_used=Bd, ws=ws, status=st)}
    B = int(Bd.item())
    rows = {}
    for kind in ("stratified", "systematic", "multinomial"):
        gpu[kind] = getattr(rs, f"resample_{kind}")(lw_d, 1, 0, ws=ws, status=st)
        a2, xo = rs.resample_and_copy(kind, lw_d, x_d, 1, 0, ws=ws, status=st)
        assert torch.equal(a2, gpu[kind]), f"{kind}: fused ancestors differ from the plain call"
        rows[kind] = xo.cpu().numpy()
    rows["metropolis"] = rs.permute_copy(gpu["metropolis"], x_d).cpu().numpy()
    gpu = {k: v.cpu().numpy() for k, v in gpu.items()}
    assert int(st.item()) == 0
    sub = np.arange(0, P, 16, dtype=np.int64)

    # one core, pinned for the measurement (the oracle is single-threaded C)
    allowed = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    pinned = allowed[0] if allowed else None
    if allowed:
        os.sched_setaffinity(0, {pinned})
    t_met, t_rest, orc = [], [], {}
    try:
        t_start = time.perf_counter()
        while True:
            t0 = time.perf_counter()
            orc["metropolis_sub"] = oracle.metropolis_subset(lw, B, 1, 0, sub)
            t1 = time.perf_counter()
            for kind in ("stratified", "systematic", "multinomial"):
                a, _, C = getattr(oracle, kind)(lw, 1, 0, want_cumw=True)
                orc[kind], orc["C"] = a, C
                oracle.ancestors_to_offspring(a)
                orc[kind + "_rows"] = oracle.permute_copy(a, x)[0]
            oracle.permute_copy(gpu["metropolis"], x)
            t_met.append(t1 - t0)
            t_rest.append(time.perf_counter() - t1)
            # a bounded sample: passes until the time budget (default 15 s) is spent
            if time.perf_counter() - t_start > args.cpu_seconds or len(t_met) >= 100:
                break
    finally:
        if allowed:
            os.sched_setaffinity(0, set(allowed))
    t_step = float(np.mean(t_met)) * P / sub.size + float(np.mean(t_rest))

    # every core: the OpenMP build of the same source
    t0 = time.perf_counter()
    a_omp, _ = oracle.metropolis_all_cores(lw, B, 1, 0)
    t_omp_met = time.perf_counter() - t0
    t0 = time.perf_counter()
    for kind in ("stratified", "systematic", "multinomial"):
        getattr(oracle, kind)(lw, 1, 0)
        oracle.ancestors_to_offspring(orc[kind])
        oracle.permute_copy_all_cores(orc[kind], x)
    r_omp, _ = oracle.permute_copy_all_cores(a_omp, x)
    t_omp_rest = time.perf_counter() - t0
    threads = omp_threads()

    parity = {"metropolis": {"B": B, "chains_compared": P,
                             "mismatches": int(np.count_nonzero(a_omp != gpu["metropolis"])),
                             "subset_mismatches": int(np.count_nonzero(
                                 orc["metropolis_sub"] != gpu["metropolis"][sub])),
                             "rows_differing": int(np.count_nonzero(
                                 (r_omp.view(np.uint32) != rows["metropolis"].view(np.uint32))
                                 .any(axis=1)))}}
    for kind in ("stratified", "systematic", "multinomial"):
        total, unexplained = count_mismatches(kind, gpu[kind], orc[kind], orc["C"], 1, 0)
        same = gpu[kind] == orc[kind]
        bad_rows = (rows[kind].view(np.uint32) != orc[kind + "_rows"].view(np.uint32)).any(axis=1)
        parity[kind] = {"mismatches": total, "unexplained": unexplained,
                        "rows_differing_where_ancestors_agree": int(np.count_nonzero(bad_rows & same))}
    return {"value": 4 * P / t_step, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": (f"{len(t_met)} passes at P={P}: stratified, systematic, multinomial, "
                       f"offspring and copies in full, Metropolis (B={B}, eq. (5)) on every "
                       f"16th chain, scaled to all P; single-threaded C oracle, one pinned core"),
            "seconds_per_step": t_step, "host_cpu": cpu_model(), "pinned_cpu": pinned,
            "allowed_cpus": len(allowed), "host_nproc": os.cpu_count(),
            "all_cores": {"value": 4 * P / (t_omp_met + t_omp_rest), "unit": "particles/s",
                          "cores": threads, "kind": "oracle (OpenMP build of the same source)",
                          "seconds_per_step": t_omp_met + t_omp_rest,
                          "metropolis_s": t_omp_met,
                          "sample": "one full step at P=2^20: Metropolis chains and copies "
                                    "on every core, the prefix resamplers single-threaded"},
            "parity": parity}


def omp_threads():
    """OpenMP's thread count for this process (what the all-core build uses)."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_get_max_threads.restype = ctypes.c_int
        return int(gomp.omp_get_max_threads())
    except OSError:
        return os.cpu_count()


def cpu_model():
    """The host CPU's model name (Linux), else the platform's description."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


if __name__ == "__main__":
    main()
