"""Autotuner for the launch parameters (they change speed, never results).

Metropolis single calls: threads per block, iterations per round (unroll),
the LDS staging threshold and lanes per chain, chosen to minimise the mean
slowdown over a set of (P, B) points (the geometric mean of each point's
time over the best time any candidate reached there, so a 4096-particle
point where LDS staging decides counts as much as a 2^20 point that takes a
thousand times longer). Batched launches: chains per work item,
unroll, LDS staging threshold and persistent grid size, chosen on a batch
shaped like the target workload. Results are stored in tuning.json next to
this file, keyed by device name and library version, and applied when the
binding is imported.

    python -m paper_1202_6163_amd.autotune [--quick] [--batch-only]

--batch-only keeps the stored single-call tuning and tunes the batched
launches alone.
"""
import argparse
import itertools
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_FILE = os.path.join(HERE, "tuning.json")


def device_key(torch, lib):
    """Architecture, compute-unit count and library version (the marketing
    name is not stable: it depends on which device-name table a process finds)."""
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
    return f"{arch}|{props.multi_processor_count}cu|v{lib.rs_version()}"


def load(torch, lib):
    """The stored tuning for this device and library version, or None."""
    try:
        rec = json.load(open(TUNING_FILE))
    except (OSError, ValueError):
        return None
    return rec.get(device_key(torch, lib))


def tune_metropolis(torch, rs, points, candidates, reps=5):
    from .timing import Graphs, pct
    from . import workloads
    G = Graphs(torch)
    data = []
    for P, B in points:
        lw = torch.from_numpy(workloads.normal_logweights(P, 1.0, 0)).cuda()
        anc = torch.empty(P, dtype=torch.int32, device="cuda")
        data.append((P, B, lw, anc))
    results = []
    for cand in candidates:
        rs.rs_metropolis_set_tuning(**cand)
        total, per = 0.0, {}
        for P, B, lw, anc in data:
            R = max(1, min(32, int(2e5 // P) + 1))
            g = G.capture(lambda: [rs.resample_metropolis(lw, B, k, 0, anc=anc) for k in range(R)])
            ms = pct(G.replay_ms([g], reps), 50) / R
            per[f"{P}:{B}"] = ms
            total += ms
        results.append((total, cand, per))
        print(f"metropolis {cand}: {total:.3f} ms", file=sys.stderr, flush=True)
    best = {k: min(r[2][k] for r in results) for k in results[0][2]}
    scored = [(float(np.exp(np.mean([np.log(per[k] / best[k]) for k in per]))), cand, per)
              for _, cand, per in results]
    scored.sort(key=lambda r: r[0])
    return scored


def tune_batch(torch, rs, instances, candidates, reps=5):
    from .batch import Batch
    from .timing import Graphs, pct
    G = Graphs(torch)
    results = []
    for cand in candidates:
        b = Batch(instances, tuning=cand)
        g = G.capture(b.run)
        results.append((pct(G.replay_ms([g], reps), 50), cand))
        print(f"batch {cand}: {results[-1][0]:.3f} ms", file=sys.stderr, flush=True)
    results.sort(key=lambda r: r[0])
    return results


def tune_batch_candidates(torch, rs, quick):
    """The batched launches' candidates on the target-shaped batch: (best,
    every result sorted by time)."""
    insts = batch_instances(torch)
    bcands = [dict(chains_per_item=c, unroll=u, lds_max_p=l, blocks=bl)
              for c, u, l, bl in itertools.product([512, 1024, 2048], [4, 8, 16],
                                                   [0, 8192, 32768], [0, 1024])]
    if quick:
        bcands = bcands[::3]
    bres = tune_batch(torch, rs, insts, bcands)
    print("batch best", bres[0][1], f"{bres[0][0]:.3f} ms", file=sys.stderr, flush=True)
    return bres[0][1], bres


def batch_instances(torch, n=1024, seed=0):
    from . import workloads
    P, sig = workloads.batch_instances(n, seed=seed)
    out = []
    for k in range(n):
        Pk = int(P[k])
        out.append(dict(
            lw=torch.from_numpy(workloads.normal_logweights(Pk, sig[k], k)).cuda(),
            anc=torch.empty(Pk, dtype=torch.int32, device="cuda"),
            kind="metropolis" if k % 2 else "stratified", B=64, seed=5, instance=k,
            x_in=torch.from_numpy(workloads.state_rows_normal(Pk, 16, k)).cuda(),
            x_out=torch.empty((Pk, 16), dtype=torch.float32, device="cuda")))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=TUNING_FILE)
    ap.add_argument("--batch-only", action="store_true")
    args = ap.parse_args()
    import torch
    import paper_1202_6163_amd.api as rs
    from ._lib import lib

    key = device_key(torch, lib)
    try:
        rec = json.load(open(args.out))
    except (OSError, ValueError):
        rec = {}
    if args.batch_only and "metropolis" not in rec.get(key, {}):
        # the stored tuning next to the package, when --out names a new file
        try:
            stored = json.load(open(TUNING_FILE)).get(key, {})
        except (OSError, ValueError):
            stored = {}
        if "metropolis" not in stored:
            raise SystemExit(f"--batch-only: no stored single-call tuning for {key}")
        rec[key] = stored

    if args.batch_only:
        entry = dict(rec[key])
        rs.rs_metropolis_set_tuning(**entry["metropolis"])
        best_b, bres = tune_batch_candidates(torch, rs, args.quick)
        entry["batch"] = best_b
        entry["batch_top"] = [dict(ms=float(t), **c) for t, c in bres[:5]]
        rec[key] = entry
        with open(args.out, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec[key]), flush=True)
        return

    points = [(1 << 12, 32), (1 << 14, 64), (1 << 16, 64), (1 << 18, 32), (1 << 20, 32),
              (1 << 20, 256)]
    blocks = [256] if args.quick else [128, 256, 512]
    unrolls = [4, 8, 16]
    ldss = [0, 16384, 40960]
    lanes = [0, 1]
    mcands = [dict(block=b, unroll=u, lds_max_p=l, lanes_per_chain=g)
              for b, u, l, g in itertools.product(blocks, unrolls, ldss, lanes)]
    mres = tune_metropolis(torch, rs, points, mcands)
    best_m = mres[0][1]
    print("metropolis best", best_m, f"{mres[0][0]:.3f} ms", file=sys.stderr, flush=True)
    rs.rs_metropolis_set_tuning(**best_m)

    best_b, bres = tune_batch_candidates(torch, rs, args.quick)
    # the staging threshold's effect: the best candidate with each threshold,
    # per point (P <= 16384 can be staged; 40960 also stages 2^15-2^16 points
    # if they fit, which they do not at the points used here)
    by_lds = {}
    for t, c, per in mres:
        by_lds.setdefault(str(c["lds_max_p"]), {"slowdown": t, **c, "ms_per_point": per})
    rec[key] = {
        "metropolis": best_m, "batch": best_b,
        "metropolis_points": [list(p) for p in points],
        "metropolis_objective": "geometric mean over points of time / best time at the point",
        "metropolis_top": [dict(slowdown=float(t), **c, ms_per_point=per)
                           for t, c, per in mres[:5]],
        "metropolis_best_per_lds_threshold": by_lds,
        "batch_top": [dict(ms=float(t), **c) for t, c in bres[:5]],
    }
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec[key]), flush=True)


if __name__ == "__main__":
    main()
