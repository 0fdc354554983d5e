#!/usr/bin/env python3
"""DCFR iterations per second on one MI355X.

A step is one full DCFR iteration of the solver (regret matching, forward
reach, fold and showdown terminals, chance averaging, backward values, regret
and average-strategy update) over one subgame whose regret and
average-strategy tables live in HBM.

Default workload: a turn subgame solved to showdown -- seeded 4-card board,
Dirichlet(1) ranges over the 1128 compatible combos, pot log-uniform in
[20, 400] and stack-to-pot ratio uniform in [1, 8] (seed 0 draws pot 166,
stacks 1006), bet sizes {33, 75, 150}% of the pot plus all-in, at most 3
bets/raises per street, FP32.

Prints one JSON line.  ``--gpus`` above 1 is refused: the solver runs on one
GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--profile-iters", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def pair_count(r0, r1, cc):
    """Number of (hand, opponent hand) pairs with mass on both sides that share no card."""
    a = np.flatnonzero(r0 > 0)
    b = np.flatnonzero(r1 > 0)
    ca = cc[a]
    cb = cc[b]
    clash = ((ca[:, 0:1] == cb[None, :, 0]) | (ca[:, 0:1] == cb[None, :, 1]) |
             (ca[:, 1:2] == cb[None, :, 0]) | (ca[:, 1:2] == cb[None, :, 1]))
    return int((~clash).sum())


def cpu_baseline(spec, r, budget_s):
    """Time the FP64 oracle on the same tree with sparse-support ranges at two
    support sizes, fit time = fixed + per_pair * pairs, and extrapolate to the
    full ranges' pair count."""
    import oracle as O
    from paper_2605_19928_amd import inputs as I

    cc = I.combo_cards()
    t = O.Tree.holdem(**spec)
    full_pairs = 2 * pair_count(r[0], r[1], cc)
    rng = np.random.default_rng(1234)
    ok = np.flatnonzero(~I.blocked_mask(spec["board"]))
    pts = []
    for k in (8, 24):
        pick = np.sort(rng.choice(ok, k, replace=False))
        rs = np.zeros_like(r)
        rs[:, pick] = r[:, pick]
        s = O.Solver(t, rs, support_only=True)
        n, t0 = 0, time.perf_counter()
        while True:
            s.iterate(1)
            n += 1
            el = time.perf_counter() - t0
            if el > budget_s / 2 or n >= 50:
                break
        pts.append((2 * pair_count(rs[0], rs[1], cc), el / n))
        del s
    (p1, t1), (p2, t2) = pts
    per_pair = max((t2 - t1) / max(p2 - p1, 1), 0.0)
    fixed = max(t1 - per_pair * p1, 0.0)
    sec_full = fixed + per_pair * full_pairs
    return {
        "value": 1.0 / sec_full,
        "unit": "iters/s",
        "cores": O.max_threads(),
        "kind": "oracle",
        "sample": (f"oracle on the same tree with random 8- and 24-combo supports per player "
                   f"({pts[0][1]:.3f} and {pts[1][1]:.3f} s/iter over {pts[0][0]} and {pts[1][0]} hand pairs); "
                   f"time = fixed + per-pair cost fitted and extrapolated to the full ranges' {full_pairs} pairs"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P

    spec, r = I.turn_config(args.seed)
    print(f"bench: building turn subgame seed={args.seed} {spec}", file=sys.stderr, flush=True)
    tree = P.Tree(**spec)
    solver = P.Solver(tree, r, P.SolverConfig(dtype=args.dtype))
    H = tree.n_hands
    units = tree.n_rows * H                       # (action row, hand) pairs
    esz = 8 if args.dtype == "f64" else 4
    alg_bytes = 4 * esz * units                   # R and S, each read and written once

    solver.iterate(args.warmup)
    solver.synchronize()
    stream = solver.stream
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    solver.iterate(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms = total_ms / args.steps
    print(f"bench: {args.steps} steps in {total_ms:.2f} ms", file=sys.stderr, flush=True)

    # per-kernel-class device time, launch by launch with HIP events
    pms, plaunch = solver.profile(args.profile_iters)
    pms = pms / args.profile_iters
    plaunch = plaunch // args.profile_iters
    names = ["bookkeeping", "forward", "terminal", "backward"]
    dom = int(np.argmax(pms))
    bwd_ms = pms[3]
    bwd_avg_us = 1e3 * bwd_ms / max(plaunch[3], 1)
    achieved = alg_bytes / (bwd_ms * 1e-3) / 1e9
    expl, br = solver.exploitability()
    print(f"bench: per-iteration kernel ms {dict(zip(names, np.round(pms, 4)))} launches {plaunch.tolist()}",
          file=sys.stderr, flush=True)

    result = {
        "metric": "DCFR ms/iter & iters/sec, flop depth-limited subgame; exploitability mbb/hand",
        "value": 1000.0 / ms,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"turn subgame to showdown, seed {args.seed}",
            "board": spec["board"], "pot": spec["pot"], "stacks": list(spec["stacks"]),
            "spr": round(spec["stacks"][0] / spec["pot"], 3),
            "bet_sizes_pct": spec["sizes"], "allin": True, "max_raises_per_street": spec["max_raises"],
            "nodes": tree.n_nodes, "decision_nodes": tree.n_decision, "chance_nodes": tree.n_chance,
            "action_rows": tree.n_rows, "hands": H, "levels": tree.n_levels,
            "state_bytes_R_S": 2 * esz * tree.n_rows * tree.n_hands_padded,
        },
        "exploitability_mbb_per_hand": expl * 100.0,
        "exploitability_after_iters": args.warmup + args.steps + args.profile_iters,
        "iteration_hbm_frac": (alg_bytes / (ms * 1e-3) / 1e9) / HBM_PEAK_GBS,
        "kernel_ms_per_iter": dict(zip(names, [float(x) for x in pms])),
        "roofline": {
            "kernel": "k_backward (value + regret + average-strategy sweep)",
            "dominant_kernel": names[dom],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": bwd_avg_us,
            "launches_per_iter": int(plaunch[3]),
            "alg_bytes_per_iter": alg_bytes,
        },
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(spec, r, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
