"""Comparison helpers for the GPU parity tests (the oracle is the reference)."""
import numpy as np

import oracle

KIND_CODE = {"stratified": oracle.KIND_STRATIFIED, "systematic": oracle.KIND_SYSTEMATIC,
             "multinomial": oracle.KIND_MULTINOMIAL}
ORACLE_FN = {"stratified": oracle.stratified, "systematic": oracle.systematic,
             "multinomial": oracle.multinomial}

# Cumulative weights: elementwise relative tolerance against the binary64
# left-to-right oracle sum (exact zero where the oracle is zero).
CUMW_RTOL = 1e-6

# What the comparisons saw, written out at the end of the session (conftest):
# the boundary mismatches of every ancestor comparison, the worst relative
# error of every cumulative-weight comparison, the hardware log's error.
REPORT = {"mismatches": [], "cumw": [], "log_u_max_rel_error": None}


def check_cumw(C_gpu, C_orc):
    C_gpu = np.asarray(C_gpu, dtype=np.float64)
    zero = C_orc == 0
    assert np.all(C_gpu[zero] == 0), "cumulative weight nonzero where the oracle's is zero"
    rel = np.abs(C_gpu[~zero] - C_orc[~zero]) / C_orc[~zero]
    worst = float(rel.max()) if rel.size else 0.0
    REPORT["cumw"].append({"P": int(C_orc.size), "worst_rel": worst})
    assert worst <= CUMW_RTOL, f"cumulative weights off by {worst:.3e} relative"
    return worst


def count_mismatches(kind, anc_gpu, anc_orc, C_orc, seed, instance):
    """(mismatches, unexplained): indices where the ancestors differ, and
    how many of those are not a draw within CUMW_RTOL of a cumulative-weight
    boundary between the two answers."""
    anc_gpu = np.asarray(anc_gpu)
    mism = np.flatnonzero(anc_gpu != anc_orc)
    if mism.size == 0:
        return 0, 0
    P = anc_orc.size
    x = oracle.draw_points(KIND_CODE[kind], P, C_orc[-1], seed, instance)
    bad = 0
    for i in mism:
        lo, hi = sorted((int(anc_gpu[i]), int(anc_orc[i])))
        if not (0 <= lo and hi < P):
            bad += 1
            continue
        bounds = C_orc[lo:hi]
        if not np.all(np.abs(x[i] - bounds) <= CUMW_RTOL * bounds):
            bad += 1
    return int(mism.size), bad


def explained_mismatches(kind, anc_gpu, anc_orc, C_orc, seed, instance):
    """Indices where the ancestors differ; each must be a draw within
    CUMW_RTOL of a cumulative-weight boundary between the two answers.
    Returns the number of (explained) mismatches."""
    anc_gpu = np.asarray(anc_gpu)
    mism = np.flatnonzero(anc_gpu != anc_orc)
    REPORT["mismatches"].append({"kind": kind, "P": int(anc_orc.size), "seed": int(seed),
                                 "instance": int(instance), "mismatches": int(mism.size)})
    if mism.size == 0:
        return 0
    P = anc_orc.size
    x = oracle.draw_points(KIND_CODE[kind], P, C_orc[-1], seed, instance)
    for i in mism:
        lo, hi = sorted((int(anc_gpu[i]), int(anc_orc[i])))
        assert 0 <= lo and hi < P, f"ancestor out of range at {i}"
        bounds = C_orc[lo:hi]  # boundaries C_j, j in [lo, hi - 1]
        ok = np.all(np.abs(x[i] - bounds) <= CUMW_RTOL * bounds)
        assert ok, (f"{kind}: unexplained ancestor mismatch at i={i}: gpu {anc_gpu[i]} "
                    f"oracle {anc_orc[i]}, x={x[i]!r}")
    return int(mism.size)


def summary():
    """Totals of REPORT per resampler kind (for the written report)."""
    by_kind = {}
    for r in REPORT["mismatches"]:
        k = by_kind.setdefault(r["kind"], {"comparisons": 0, "particles": 0, "mismatches": 0,
                                           "max_in_one": 0})
        k["comparisons"] += 1
        k["particles"] += r["P"]
        k["mismatches"] += r["mismatches"]
        k["max_in_one"] = max(k["max_in_one"], r["mismatches"])
    cum = REPORT["cumw"]
    return {"by_kind": by_kind,
            "cumw_comparisons": len(cum),
            "cumw_worst_rel": max((c["worst_rel"] for c in cum), default=None),
            "log_u_max_rel_error": REPORT["log_u_max_rel_error"],
            "note": "every mismatch counted here was checked to be a draw within 1e-6 "
                    "relative of a cumulative-weight boundary between the two answers"}
