"""Benchmark of the resampling stage on one MI355X.

Step (the timed unit): one pass of the whole resampling path over one batch
of P = 2^20 particles with log-weights N(0, sigma^2) (sigma = 1) and D = 4
binary32 state rows: the Metropolis (B = 32), stratified, systematic and
multinomial resamplers, each in the paper's output form (offspring for
stratified and systematic, written in the same pass as the ancestors the copy
needs; ancestors for the other two) and the ancestor-indexed state copy
(in the stratified and systematic fill itself, a launch of its own after the
other two). Every step uses the next of several rotating
input/output buffer sets whose total exceeds the 256 MB Infinity Cache, so
the step reads its inputs from HBM. value = resampled particles per second
(4 P per step) at the p99 step time.

Beside it the JSON line carries:
  roofline      the dominant kernel of the step against its ceiling;
  roofline_hbm  the stratified resample + state copy path against HBM;
  sweep         per sigma and P, p50/p99 particles/s of every resampler
                (Metropolis at each B), with and without the copy, the
                accuracy metric sum_i (o_i/P - w_i/W)^2, the ESS, eq. (5)'s B
                and the Metropolis-vs-stratified crossover (warm cache);
  dirichlet     Sec. 3's experiment: Dirichlet weights, P = 256 .. 65536,
                error and per-call time of every resampler and the
                sorted-weight variants;
  batched       1024 independent instances in one batched launch against
                per-instance calls;
  filter        the bootstrap filter (P = 2^18, D = 8, T = 200) against the
                Kalman log-likelihood;
  pmcmc         particle marginal Metropolis-Hastings with batched filters;
  serving       Poisson arrivals at 2000 req/s: latency percentiles;
  cpu_baseline  the CPU oracle on a bounded sample of the same step.
"""
import argparse
import hashlib
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
# VALU issue rate from the unit counts: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
# Algorithmic VALU slots per Metropolis iteration: half a Philox4x32-10 block
# (10 rounds x (two quarter-rate 32x32->64 multiplies + two 3-input xors)
# / 2 = 50) plus the quarter-rate high-word multiply of the index map (4).
METRO_SLOTS_PER_ITER = 54.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--P", type=int, default=1 << 20)
    ap.add_argument("--D", type=int, default=4)
    ap.add_argument("--sigma", type=float, default=1.0)
    ap.add_argument("--B", type=int, default=32)
    ap.add_argument("--sets", type=int, default=8, help="rotating buffer sets (cold HBM)")
    ap.add_argument("--reps", type=int, default=40, help="timed calls per sweep point")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--sweep-P", type=str, default="12,14,16,18,20")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-filter", action="store_true")
    ap.add_argument("--no-dirichlet", action="store_true")
    ap.add_argument("--dirichlet-R", type=int, default=50)
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="seconds of Poisson arrivals at 2000 req/s (0: skip; the full run is 60)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only", type=str, default="", help="time one kernel (for profiling)")
    ap.add_argument("--out", type=str, default="")
    return ap.parse_args()


from paper_1202_6163_amd.timing import Graphs, pct  # noqa: E402


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU sharding is "
                                   "a design only, not built", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1202_6163_amd.api as rs
    from paper_1202_6163_amd import workloads

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    P, D, B, sigma = args.P, args.D, args.B, args.sigma
    dev = torch.device("cuda", 0)

    # ------------------------------------------------ rotating cold buffer sets
    sets = []
    for s in range(args.sets):
        lw = torch.from_numpy(workloads.normal_logweights(P, sigma, s)).to(dev)
        x = torch.from_numpy(workloads.state_rows_normal(P, D, s)).to(dev)
        sets.append(dict(lw=lw, x=x, anc=torch.empty(P, dtype=torch.int32, device=dev),
                         off=torch.empty(P, dtype=torch.int32, device=dev),
                         xo=torch.empty_like(x)))
    ws = rs.workspace(P, rs.MULTINOMIAL, dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    set_bytes = sum(t.numel() * t.element_size() for t in sets[0].values())

    def step(bs, seed, inst):
        # Each resampler in the paper's output form (Sec. 2: stratified and
        # systematic give offspring, multinomial and Metropolis ancestors),
        # and the ancestor-indexed state copy. Stratified and systematic copy
        # the rows in their own fill (resample_and_copy: the same ancestors,
        # offspring and rows, one launch fewer, faster at this size);
        # Metropolis and multinomial run the copy as its own launch, which is
        # faster for them (both forms are timed and reported).
        rs.resample_metropolis(bs["lw"], B, seed, inst, anc=bs["anc"], status=status)
        rs.permute_copy(bs["anc"], bs["x"], x_out=bs["xo"], status=status)
        for kind in ("stratified", "systematic"):
            rs.resample_and_copy(kind, bs["lw"], bs["x"], seed, inst, anc=bs["anc"],
                                 off=bs["off"], x_out=bs["xo"], ws=ws, status=status)
        rs.resample_multinomial(bs["lw"], seed, inst, anc=bs["anc"], ws=ws, status=status)
        rs.permute_copy(bs["anc"], bs["x"], x_out=bs["xo"], status=status)

    if args.only:
        # profiling mode: plain launches of one kernel family on the cold sets
        big = torch.empty(1 << 24, dtype=torch.float32, device=dev)  # 64 MiB
        big_out = torch.empty_like(big)
        only = {"metropolis": lambda bs, k: rs.resample_metropolis(bs["lw"], B, k, 0, anc=bs["anc"]),
                "copycal": lambda bs, k: big_out.copy_(big),
                "stratified": lambda bs, k: rs.resample_stratified(bs["lw"], k, 0, anc=bs["anc"], ws=ws,
                                                                   off=bs["off"]),
                "multinomial": lambda bs, k: rs.resample_multinomial(bs["lw"], k, 0, anc=bs["anc"],
                                                                     ws=ws),
                "copy": lambda bs, k: rs.permute_copy(bs["anc"], bs["x"], x_out=bs["xo"]),
                "step": lambda bs, k: step(bs, k, 0)}[args.only]
        for bs in sets:
            rs.resample_stratified(bs["lw"], 1, 0, anc=bs["anc"], ws=ws)
        for k in range(args.warmup):
            only(sets[k % len(sets)], k)
        # HIP events around the timed calls (back to back on one stream), so a
        # profiler's per-kernel average can be set beside the same run's
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(args.warmup, args.warmup + args.steps):
            only(sets[k % len(sets)], k)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / max(args.steps, 1)
        print(f"profiled {args.only}: {args.warmup + args.steps} calls; {us:.2f} us per timed call "
              f"(HIP events, {args.steps} calls)", flush=True)
        return

    G = Graphs(torch)
    step_graphs = [G.capture(lambda bs=bs, k=k: step(bs, 1000 + k, 0)) for k, bs in enumerate(sets)]
    G.replay_ms(step_graphs, max(args.warmup, 1))

    # ------------------------------------------------ timed steps (cold)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms = G.replay_ms(step_graphs, args.steps)
    wall = time.perf_counter() - t0
    assert int(status.item()) == 0, f"status flags {int(status.item())}"
    p99 = pct(step_ms, 99)
    value = 4 * P / (p99 * 1e-3)

    # ------------------------------------------------ per-kernel rooflines (cold)
    def time_calls(fn, per_graph=None, replays=8):
        """Mean GPU time of one call: graphs of one call per buffer set."""
        n_sets = len(sets)
        g = G.capture(lambda: [fn(bs, k) for k, bs in enumerate(sets)])
        ms = G.replay_ms([g], replays)
        return [m / n_sets for m in ms]

    for bs in sets:  # sorted ancestors for the copy
        rs.resample_stratified(bs["lw"], 7, 0, anc=bs["anc"], ws=ws)
    copy_ms = time_calls(lambda bs, k: rs.permute_copy(bs["anc"], bs["x"], x_out=bs["xo"]))
    strat_ms = time_calls(lambda bs, k: rs.resample_stratified(bs["lw"], k, 0, anc=bs["anc"], ws=ws,
                                                               off=bs["off"]))
    metro_ms = time_calls(lambda bs, k: rs.resample_metropolis(bs["lw"], B, k, 0, anc=bs["anc"]))
    multi_ms = time_calls(lambda bs, k: rs.resample_multinomial(bs["lw"], k, 0, anc=bs["anc"], ws=ws))
    syst_ms = time_calls(lambda bs, k: rs.resample_systematic(bs["lw"], k, 0, anc=bs["anc"], ws=ws,
                                                              off=bs["off"]))
    # the copy above used sorted ancestors; the sweep reports unsorted ones too
    for bs in sets:
        rs.resample_stratified(bs["lw"], 7, 0, anc=bs["anc"], ws=ws)
    means = {"metropolis": np.mean(metro_ms), "stratified": np.mean(strat_ms),
             "systematic": np.mean(syst_ms), "multinomial": np.mean(multi_ms),
             "permute_copy": np.mean(copy_ms)}
    fused_means = {}
    for kind in ("metropolis", "stratified", "systematic", "multinomial"):
        fused_means[kind] = float(np.mean(time_calls(
            lambda bs, k, kind=kind: rs.resample_and_copy(
                kind, bs["lw"], bs["x"], k, 0, B=B, anc=bs["anc"],
                off=bs["off"] if kind in ("stratified", "systematic") else None, x_out=bs["xo"],
                ws=None if kind == "metropolis" else ws))))
    dominant = max(means, key=means.get)
    iters = float(P) * B
    traffic = load_traffic(dominant)
    if dominant == "metropolis":
        achieved = iters * METRO_SLOTS_PER_ITER / (means["metropolis"] * 1e-3) / 1e12
        peak = VALU_SLOTS_PER_S / 1e12
        roofline = {"bound": "alu", "achieved": achieved, "peak": peak,
                    "unit": "TVALU-slot/s", "frac": achieved / peak, "traffic": traffic,
                    "limiter": "random 4-byte L2 gathers of the proposed weights: see "
                               "measured_ceilings (the VALU model prices Philox high)",
                    "kernel": "metropolis_kernel", "avg_launch_us": means["metropolis"] * 1e3,
                    "units_per_launch": {"chain_iterations": iters},
                    "algorithmic_per_unit": {"valu_slots": METRO_SLOTS_PER_ITER}}
    else:
        per = {"stratified": 16, "systematic": 16, "multinomial": 24,
               "permute_copy": 4 + 8 * D}[dominant]
        achieved = per * P / (means[dominant] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dominant,
                    "avg_launch_us": means[dominant] * 1e3}
    roofline["measured_ceilings"] = ceilings(torch, rs, G, sets[0]["lw"], iters / (means["metropolis"] * 1e-3))
    copy_gbs = (4 + 8 * D) * P / (np.mean(copy_ms) * 1e-3) / 1e9
    strat_gbs = 16 * P / (np.mean(strat_ms) * 1e-3) / 1e9
    path_gbs = (16 + 4 + 8 * D) * P / ((np.mean(copy_ms) + np.mean(strat_ms)) * 1e-3) / 1e9
    roofline_hbm = {
        "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "permute_copy": {"achieved": copy_gbs, "frac": copy_gbs / HBM_PEAK_GBS,
                         "bytes_per_particle": 4 + 8 * D, "avg_launch_us": np.mean(copy_ms) * 1e3},
        "stratified": {"achieved": strat_gbs, "frac": strat_gbs / HBM_PEAK_GBS,
                       "bytes_per_particle": 16, "avg_call_us": np.mean(strat_ms) * 1e3,
                       "launches": 3, "outputs": "ancestors and offspring"},
        "stratified_plus_copy": {"achieved": path_gbs, "frac": path_gbs / HBM_PEAK_GBS,
                                 "bytes_per_particle": 20 + 8 * D},
    }

    roofline_hbm["by_P"] = hbm_by_P(torch, rs, G, D)
    out = {
        "metric": "resampled particles/s at P=2^20 (Metropolis B vs stratified) by weight var; p99",
        "value": value, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": float(np.mean(step_ms)),
        "p50_ms_per_step": pct(step_ms, 50), "p99_ms_per_step": p99,
        "wall_s_timed": wall, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 weights / f64 prefix sums / u32 Philox",
        "data": "synthetic", "config": {
            "workload": "resampler sweep point P=2^20, lw ~ N(0, 1), D=4 state copy; step = "
                        "Metropolis(B=32) + stratified + systematic + multinomial, each with "
                        "the state copy (fused into the stratified/systematic fill, which "
                        "writes ancestors, offspring and rows in one pass); cold HBM "
                        "(rotating buffer sets)",
            "P": P, "D": D, "sigma": sigma, "B": B, "buffer_sets": args.sets,
            "set_bytes": set_bytes, "parallelism": "single GPU"},
        "per_call_ms_cold": {k: float(v) for k, v in means.items()},
        "per_call_ms_cold_with_fused_copy": fused_means,
        "roofline": roofline, "roofline_hbm": roofline_hbm,
        "device": torch.cuda.get_device_name(0),
    }
    if not args.no_sweep:
        out["sweep"] = sweep(torch, rs, workloads, args)
    if not args.no_batch:
        out["batched"] = batched(torch, rs, workloads, args)
    if not args.no_dirichlet:
        out["dirichlet"] = dirichlet(torch, rs, workloads, args)
    if not args.no_filter:
        out["filter"] = filter_run(torch, workloads, args)
        out["pmcmc"] = pmcmc_run(torch, workloads, args)
    if args.serve_seconds > 0:
        out["serving"] = serving(torch, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, workloads)
    line = json.dumps(out)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)


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


def hbm_by_P(torch, rs, G, D):
    """Stratified (ancestors + offspring) + state copy against HBM at growing P
    (cold buffer sets): the fixed launch latency of the three dependent
    launches is amortised as P grows."""
    dev = torch.device("cuda", 0)
    res = {}
    for lg in (22, 24):
        P = 1 << lg
        nsets = 2 if lg >= 24 else 4
        sets = [dict(lw=torch.randn(P, device=dev), x=torch.randn(P, D, device=dev),
                     xo=torch.empty(P, D, device=dev),
                     anc=torch.empty(P, dtype=torch.int32, device=dev),
                     off=torch.empty(P, dtype=torch.int32, device=dev)) for _ in range(nsets)]
        ws = rs.workspace(P, rs.MULTINOMIAL, dev)

        def body(copy):
            for k, bs in enumerate(sets):
                rs.resample_stratified(bs["lw"], k, 0, anc=bs["anc"], ws=ws, off=bs["off"])
                if copy:
                    rs.permute_copy(bs["anc"], bs["x"], x_out=bs["xo"])
        entry = {}
        for name, copy, bpp in (("stratified", False, 16), ("stratified_plus_copy", True, 20 + 8 * D)):
            g = G.capture(lambda copy=copy: body(copy))
            G.replay_ms([g], 2)
            us = float(np.median(G.replay_ms([g], 6))) * 1e3 / nsets
            gbs = bpp * P / (us * 1e-6) / 1e9
            entry[name] = {"us": us, "achieved": gbs, "frac": gbs / HBM_PEAK_GBS,
                           "bytes_per_particle": bpp}
        res[f"2^{lg}"] = entry
        del sets
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


# The sources each kernel family is compiled from (what invalidates its counters).
KERNEL_SOURCES = {
    "metropolis": ["metropolis.hip", "metropolis_impl.h", "common.h", "launch.h"],
    "permute_copy": ["misc.hip", "common.h", "launch.h"],
    "stratified": ["prefix.hip", "prefix_impl.h", "prefix.h", "analysis.h", "common.h", "launch.h"],
    "multinomial": ["prefix.hip", "prefix_impl.h", "prefix.h", "analysis.h", "common.h", "launch.h"],
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

            def measure(call, with_copy):
                R = max(1, min(64, int(2e5 // P) + 1))  # calls per graph (>= ~50 us of work)

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
                r = measure(call, False)
                r["with_copy"] = measure(call, True)
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
    sorted-weight multinomial and systematic. Per-call times are eager calls
    (events around R back-to-back calls, host dispatch included) for every
    resampler, since the sort inside the sorted variants is not
    graph-capturable; the others also get the GPU time of a graph of R calls."""
    dev = torch.device("cuda", 0)
    R = args.dirichlet_R
    G = Graphs(torch)
    out = {"note": "us_per_call: eager per-call time (host dispatch included); "
                   "us_per_call_graph: GPU time per call in a graph of R calls (not for the "
                   "sorted variants); error averaged over R resamplings with different seeds",
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
                if not name.endswith("_sorted"):
                    g = G.capture(lambda call=call: [call(900 + k) for k in range(R)])
                    ms = G.replay_ms([g], 3)
                    point["resamplers"][name]["us_per_call_graph"] = pct(ms, 50) * 1e3 / R
            out["points"].append(point)
            print(f"dirichlet P={P} alpha={alpha}: " + ", ".join(
                f"{k} {v['us_per_call']:.1f}us ({v.get('us_per_call_graph', float('nan')):.1f} in a graph)"
                for k, v in point["resamplers"].items()),
                file=sys.stderr, flush=True)
    return out


def batched(torch, rs, workloads, args):
    """1024 instances, P log-uniform in [2^8, 2^16], sigma in [0.25, 3],
    Metropolis B = 64 and stratified alternating, D = 16: one batched graph
    replay against the same work as per-instance calls (resample +
    permute_copy) captured in one graph, and launched one by one."""
    from paper_1202_6163_amd.batch import Batch
    dev = torch.device("cuda", 0)
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
    return {"instances": len(P), "particles": total, "D": 16,
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
    """Poisson arrivals at 2000 req/s, P log-uniform in [2^10, 2^20], sigma in
    [0.5, 4], D in {1, 16}, Metropolis B = 64 or stratified, resident on the
    device, admitted by footprint, continuously batched on 4 streams."""
    from paper_1202_6163_amd.serve import GpuExecutor, make_requests, serve, summarize
    reqs = make_requests(rate=2000.0, duration=args.serve_seconds, seed=0)
    ex = GpuExecutor(n_streams=4)
    sched = serve(reqs, ex, budget_bytes=32 << 30, max_batch=256)
    s = summarize(sched, args.serve_seconds)
    s.update({"rate_req_per_s": 2000.0, "seconds": args.serve_seconds,
              "budget_bytes": 32 << 30, "streams": 4})
    return s


def cpu_baseline(args, workloads):
    """The oracle (single-threaded C, as committed) on a bounded sample of the
    step: the same four resamplers + offspring + copy at P = 2^20, timed over
    whole steps until about --cpu-seconds of CPU time."""
    import oracle
    P, D, B = args.P, args.D, args.B
    lw = workloads.normal_logweights(P, args.sigma, 0)
    x = workloads.state_rows_normal(P, D, 0)
    # one core, pinned for the measurement (the oracle is single-threaded C)
    allowed = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    pinned = None
    if allowed:
        pinned = allowed[0]
        os.sched_setaffinity(0, {pinned})
    times = []
    try:
        t_start = time.perf_counter()
        while True:
            t0 = time.perf_counter()
            for kind in ("metropolis", "stratified", "systematic", "multinomial"):
                if kind == "metropolis":
                    anc, _ = oracle.metropolis(lw, B, 1, 0)
                else:
                    anc, _ = getattr(oracle, kind)(lw, 1, 0)
                oracle.ancestors_to_offspring(anc)
                oracle.permute_copy(anc, x)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_start > args.cpu_seconds or len(times) >= 20:
                break
    finally:
        if allowed:
            os.sched_setaffinity(0, set(allowed))
    t = float(np.mean(times))
    return {"value": 4 * P / t, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} full steps at P={P} (4 resamplers + offspring + copy, "
                      f"Metropolis B={B}), single-threaded C oracle",
            "seconds_per_step": t, "host_cpu": cpu_model(), "pinned_cpu": pinned,
            "allowed_cpus": len(allowed), "host_nproc": os.cpu_count()}


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
