"""The benchmark's last stdout line (CPU only): built from a full results
record with every section present, at the magnitudes a run at P = 2^20
produces, it stays under 4 KB and keeps every key of the JSON contract,
the roofline with its traffic and the CPU baseline."""
import json

import pytest

bench = pytest.importorskip("bench")


def full_record():
    per_call = {name: {"us": 21.123456, "us_p50": 21.1, "bytes_touched_per_replay": 541065216,
                       "cold": True}
                for name in ("metropolis", "metropolis_adaptive", "metropolis_B32", "stratified",
                             "systematic", "multinomial", "permute_copy_random",
                             "permute_copy_sorted", "stratified_and_copy", "systematic_and_copy",
                             "multinomial_and_copy", "metropolis_and_copy",
                             "stratified_and_copy_onepass")}
    hbm = {k: {"frac": 0.2234567, "us": 28.123456, "bytes_per_particle": 48}
           for k in ("permute_copy", "stratified", "stratified_plus_copy", "stratified_and_copy",
                     "systematic_and_copy", "single_pass")}
    serve_pt = {"rate_req_per_s": 2000.0, "p50_latency_ms": 0.27712345, "p99_latency_ms": 2.3312345,
                "particles_per_s": 303140000.123, "mean_batch": 1.0831234, "requests": 120000}
    return {
        "metric": "resampled particles/s at P=2^20 (Metropolis B vs stratified) by weight var; p99",
        "value": 1572900000.0123, "unit": "particles/s", "n_gpus": 1, "steps": 50, "warmup": 10,
        "ms_per_step": 1.5802419948577882, "p50_ms_per_step": 1.5143799781799316,
        "p99_ms_per_step": 2.6666672635078417, "wall_s_timed": 0.08, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 log-weights / f64 prefix sums / u32 Philox",
        "data": "synthetic",
        "config": {"workload": bench.WORKLOAD, "P": 1 << 20, "D": 4, "sigma": 1.0,
                   "metropolis_B": "eq. (5), eps=0.01 (B=257 for buffer set 0)",
                   "buffer_sets": 43, "state_pairs": 16, "parallelism": "single GPU"},
        "step": {"p50_ms": 1.514, "p99_ms": 2.667, "mean_ms": 1.58},
        "step_fixed_B": {"B": 32, "B_eq5": 257, "converged": False, "p50_ms": 0.2748,
                         "p99_ms": 0.2797262033820152, "particles_per_s_p99": 1.49943e10},
        "per_call": per_call,
        "roofline": {"bound": "l2", "achieved": 258.8123456, "peak": 307.2, "unit": "Greq/s",
                     "frac": 0.84243123, "traffic": 57090558.64483801,
                     "kernel": "metropolis_kernel", "avg_launch_us": 1041.3123,
                     "alu_view": {"frac": 0.3554123},
                     "measured_ceilings": {"random_gather_per_s": 249050000000.123,
                                           "frac_of_measured_ceiling": 1.0391234}},
        "roofline_hbm": hbm,
        "sweep": {"crossover_sigma_by_P": {"4096": 0.5, "16384": 0.5, "65536": 0.25,
                                           "262144": None, "1048576": None}},
        "batched": {"batched_ms_p50": 1.4446123, "speedup_vs_per_instance_graph": 10.365123},
        "minimal_copy": {f"D{D}": {"permute_copy_us": 20.2156, "inplace_us": 20.4867,
                                   "anc_to_off_plus_inplace_us": 66.6317,
                                   "anc_to_off_ws_plus_inplace_us": 42.3794,
                                   "bytes_ratio_vs_permute_copy": 0.7887069}
                         for D in (4, 16)},
        "serving": {name: dict(serve_pt) for name in (
            "config_load", "small_8k", "small_8k_per_request_launches", "small_16k",
            "small_16k_per_request_launches")},
        "cpu_baseline": {"value": 855464.3604263195, "unit": "particles/s", "cores": 1,
                         "kind": "oracle",
                         "sample": "27 passes at P=1048576: stratified, systematic, multinomial, "
                                   "offspring and copies in full, Metropolis (B=257, eq. (5)) on "
                                   "every 16th chain, scaled to all P; single-threaded C oracle, "
                                   "one pinned core",
                         "all_cores": {"value": 6898386.98652603, "cores": 16},
                         "parity": {k: {"mismatches": 0, "unexplained": 0,
                                        "rows_differing_where_ancestors_agree": 0}
                                    for k in ("metropolis", "stratified", "systematic",
                                              "multinomial")}},
    }


def test_headline_is_compact_and_keeps_the_contract():
    h = bench.headline(full_record(), "results/bench_full.json")
    line = json.dumps(h)
    assert len(line) <= 4000, len(line)
    assert "\n" not in line
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline"):
        assert key in h, key
    assert h["config"]["workload"] == bench.WORKLOAD
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in h["roofline"], key
    assert abs(h["roofline"]["frac"] - h["roofline"]["achieved"] / h["roofline"]["peak"]) < 1e-3
    for key in ("value", "unit", "cores", "kind", "sample"):
        assert key in h["cpu_baseline"], key
    assert h["cpu_baseline"]["kind"] == "oracle"
    # the serving and batching summaries fit beside them (per-call times go first)
    assert "serving" in h and "batched" in h and "minimal_copy" in h
    assert h["value"] == pytest.approx(4 * (1 << 20) / (h["p99_ms_per_step"] * 1e-3), rel=1e-3)
