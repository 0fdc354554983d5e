#!/usr/bin/env python3
"""DCFR iterations per second on one MI355X.

A step is one full DCFR iteration of the solver over one subgame, with every
stage on the GPU: regret matching and forward reach, fold terminals, exact
all-in leaves, the batched leaf-network evaluation (input build, bf16 MFMA
GEMMs, chance-weighted combine), backward values, regret and
average-strategy updates.

Default workload (``--workload flop``): the depth-limited flop subgame --
seeded 3-card board, Dirichlet(1) ranges over the 1176 compatible combos, pot
100, stacks 400, bet sizes {33, 75}% of the pot plus all-in, at most 3
bets/raises, leaves at the turn card: 36 decision nodes, 21 network leaves x
49 turn cards = 1029 network rows per iteration, 14 exact all-in leaves.
Leaf network 2705 -> 4 x 1536 -> 2652 (ReLU), bf16 weights, FP32 accumulate;
random He-initialised weights (no trained weights ship with the benchmark).
Tree arithmetic FP32.

Secondary workload (``--workload turn``, and reported inside the flop line
as ``tree_sweep``): a turn subgame solved to showdown -- seeded 4-card board,
Dirichlet(1) ranges, pot 166, stacks 1006 (seed 0 of pot log-uniform in
[20, 400] and stack-to-pot uniform in [1, 8]), sizes {33, 75, 150}% +
all-in, at most 3 per street: 77,529 nodes, 74,312 action rows, FP32.  Its
685 MB of regret and average-strategy state is the HBM-bound part.

Batch workload (``--workload batch``, and ``batch`` inside the flop line):
256 independent subgames, 179 river + 77 turn, each with its own board,
ranges, pot, stack and bet abstraction, redrawn until 10-2000 nodes; one
forest advanced by one graph replay per iteration after the launch-schedule
autotuner, against the same subgames solved one at a time.

Flop batch (``--workload flop-batch``, and ``flop_batch`` inside the flop
line): 8 and 32 depth-limited flops of the default abstraction, each with its
own board and ranges, in one forest with one leaf network (1536 x 4), so
every iteration sends all their (leaf, next card) rows through the same GEMMs.

Training data (``--workload datagen`` only): random turn subgames of the leaf
network's training recipe solved by the batched plain solver to 1000
iterations each (a sample of ``--datagen-subgames``), with the rate and the
time the recipe's 100k subgames would take.

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
BF16_PEAK_TFLOPS = 2500.0

# HBM bytes measured with rocprofv3 hardware counters (FETCH_SIZE and
# WRITE_SIZE, one run each, scaled by the same counters over a 1 GiB copy;
# tables and commands in profiles/*_hbm_counters.md).  They describe the
# kernels as they were measured; a changed kernel needs a new measurement.
MEASURED_TRAFFIC = {
    # hidden-layer GEMMs (bias + ReLU; k_gemm_nt<BM,BN,1,KS,PF> and
    # k_gemm_direct<4,KSPLIT,..>), 1029 rows: per launch for each forward tile
    # (PCFR_TILE_*), averaged over that tile's dispatches in the counter run
    # (the autotuner's trials on the input and hidden layers): (read, write) bytes
    "gemm_hidden_by_tile": {0: (28313758, 3342336), 1: (27523328, 3342336), 2: (27516928, 3342336),
                            3: (27592704, 3342336), 4: (31257147, 3342336), 5: (27551872, 3342336),
                            6: (27490667, 3342336), 7: (27545685, 3342336), 8: (23071744, 3342336),
                            9: (23026688, 3342336), 10: (23012096, 3342336)},
    # k_backward<float,0,*> + k_backward_fused over one iteration of the
    # seed-0 turn subgame (all backward launches)
    "turn_backward_iteration": 2442259200,
    # k_backward<float,0,*> + k_backward_fused over the last (tuned) iteration
    # of the seed-0 256-subgame forest
    "batch_backward_iteration": 4030041920,
}
CLASSES = ["bookkeeping", "forward", "terminal", "backward", "leaves", "leaf_gemm_hidden", "leaf_gemm_out"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", default="flop", choices=["flop", "turn", "batch", "flop-batch", "preflop", "datagen"])
    ap.add_argument("--datagen-subgames", type=int, default=1024,
                    help="--workload datagen: random turn subgames solved (a sample of the 100k of the recipe)")
    ap.add_argument("--datagen-iters", type=int, default=1000, help="--workload datagen: solver iterations each")
    ap.add_argument("--batch-flops", type=int, default=32, help="flops per forest for --workload flop-batch")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--profile-iters", type=int, default=5)
    ap.add_argument("--no-secondary", action="store_true", help="skip the turn and batch measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip training a leaf network and the exact flop solve")
    ap.add_argument("--no-one-at-a-time", action="store_true",
                    help="batch workload: skip timing the subgames one at a time")
    ap.add_argument("--no-persistent", action="store_true",
                    help="batch workload: skip timing the persistent cooperative launch")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-mb", type=int, default=0,
                    help="first run a plain elementwise kernel over this many MiB (reads it once, writes it "
                         "once) so hardware byte counters can be scaled against a known size")
    return ap.parse_args()


def log(*a):
    print("bench:", *a, file=sys.stderr, flush=True)


def pair_count(r0, r1, cc):
    """Number of (hand, opponent hand) pairs with mass on both sides that share no card."""
    a = np.flatnonzero(r0 > 0)
    b = np.flatnonzero(r1 > 0)
    ca, cb = cc[a], cc[b]
    clash = ((ca[:, 0:1] == cb[None, :, 0]) | (ca[:, 0:1] == cb[None, :, 1]) |
             (ca[:, 1:2] == cb[None, :, 0]) | (ca[:, 1:2] == cb[None, :, 1]))
    return int((~clash).sum())


def history_visits(tree, spec, r):
    """Per-iteration history visits in the paper's sense: over every node, the
    number of (hand, opponent hand) pairs with mass on both sides that share
    no card with each other or with the node's board."""
    from paper_2605_19928_amd import inputs as I

    cc = I.combo_cards()
    e = tree.export()
    n = len(e["type"])
    dealt = [()] * n
    for v in range(1, n):
        c = int(e["chance_card"][v])
        dealt[v] = dealt[e["parent"][v]] + ((c,) if c >= 0 else ())
    groups = {}
    for d in dealt:
        groups[d] = groups.get(d, 0) + 1
    total = 0
    for d, cnt in groups.items():
        keep = np.ones(len(cc), dtype=bool)
        for c in d:
            keep &= (cc[:, 0] != c) & (cc[:, 1] != c)
        total += cnt * pair_count(r[0] * keep, r[1] * keep, cc)
    return total


def copy_ceiling_gbs(mib=1024, reps=10):
    """HBM copy bandwidth of the box: a device-to-device copy of `mib` MiB
    (read once, written once), event-timed."""
    import torch

    x = torch.ones(mib * (1 << 18), dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / reps * 1e-3
    del x, y
    return 2.0 * mib * (1 << 20) / sec / 1e9


def cpu_baseline(spec, r, budget_s, leaf_params=None):
    """Time the FP64 oracle on the full workload: whole iterations on the same
    tree and full ranges (one warm-up iteration, then as many as fit in
    budget_s, at least two).  With a leaf network each iteration first
    refreshes the leaf table (leaf inputs + FP64 forward of every leaf row)
    from the current reach, then walks the tree; both parts are timed."""
    import oracle as O
    from oracle import mlp

    t = O.Tree.holdem(**spec)
    e = t.export()
    leaves = np.flatnonzero(e["type"] == O.T_LEAF)
    eff = min(spec["stacks"])
    cores = O.max_threads()
    if leaf_params is None:
        return cpu_baseline_ladder(t, r, spec, budget_s, cores)
    s = O.Solver(t, r)

    def refresh():
        if leaf_params is None or not len(leaves):
            return
        reach = s.reach_current()
        ev = np.zeros((len(leaves), 2, 52, 1326))
        for li, node in enumerate(leaves):
            c = e["contrib"][node][0]
            cards, X = mlp.leaf_inputs(reach[node], spec["board"], 2 * c, spec["pot"] // 2 + eff - c, 2705)
            Y = mlp.forward(leaf_params, X, emulate_bf16=True)
            for kk, card in enumerate(cards):
                ev[li, 0, card] = Y[kk, :1326]
                ev[li, 1, card] = Y[kk, 1326:]
        s.set_leaf_table(ev)

    refresh()
    s.iterate(1, threads=cores)                 # warm-up (allocation)
    net_s = walk_s = 0.0
    n, t0 = 0, time.perf_counter()
    while True:
        ta = time.perf_counter()
        refresh()
        tb = time.perf_counter()
        s.iterate(1, threads=cores)
        tc = time.perf_counter()
        net_s += tb - ta
        walk_s += tc - tb
        n += 1
        if n >= 2 and time.perf_counter() - t0 > budget_s:
            break
    sec = (time.perf_counter() - t0) / n
    # one more iteration on a single thread (the oracle's OpenMP walk and the
    # FP64 network refresh's BLAS both held to one thread)
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):
        ta = time.perf_counter()
        refresh()
        tb = time.perf_counter()
        s.iterate(1, threads=1)
        tc = time.perf_counter()
    single = {"value": 1.0 / (tc - ta), "unit": "iters/s", "cores": 1,
              "parts_s_per_iter": {"leaf_network": tb - ta, "walk": tc - tb},
              "sample": f"one oracle iteration of the full workload on one thread: {tc - ta:.3f} s"}
    del s
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": 1.0 / sec,
        "unit": "iters/s",
        "cores": cores,
        "kind": "oracle",
        "host_cpu": cpu_model, "host_nproc": os.cpu_count(),
        "parts_s_per_iter": {"leaf_network": net_s / n, "walk": walk_s / n},
        "sample": (f"{n} oracle iterations of the full workload (same tree, full ranges) after one warm-up, "
                   f"{sec:.3f} s each: FP64 leaf-network refresh {net_s / n:.3f} s + tree walk "
                   f"{walk_s / n:.3f} s on {cores} threads"),
        "single_thread": single,
    }


def cpu_baseline_ladder(t, r, spec, budget_s, cores):
    """For trees whose full oracle iteration takes minutes (the turn): one
    iteration at random supports of 24, 48, 96, ... combos per player until
    one takes an eighth of budget_s or the support is full; seconds per
    iteration extrapolated linearly in hand pairs from the last two points."""
    import oracle as O
    from paper_2605_19928_amd import inputs as I

    cc = I.combo_cards()
    ok = np.flatnonzero(~I.blocked_mask(spec["board"]))
    full_pairs = 2 * pair_count(r[0], r[1], cc)
    pts, k, t_all = [], 24, time.perf_counter()
    while True:
        pick = np.sort(np.random.default_rng(1234 + k).choice(ok, min(k, len(ok)), replace=False))
        rs = np.zeros_like(r)
        rs[:, pick] = r[:, pick]
        s = O.Solver(t, rs, support_only=True)
        s.iterate(1, threads=cores)             # warm-up (allocation)
        t0 = time.perf_counter()
        s.iterate(1, threads=cores)
        pts.append((2 * pair_count(rs[0], rs[1], cc), time.perf_counter() - t0))
        del s
        if k >= len(ok) or pts[-1][1] > budget_s / 8 or time.perf_counter() - t_all > budget_s:
            break
        k *= 2
    if len(pts) == 1 or pts[-1][0] >= full_pairs:
        sec = pts[-1][1] * full_pairs / max(pts[-1][0], 1)
    else:
        (p1, t1), (p2, t2) = pts[-2], pts[-1]
        per_pair = max((t2 - t1) / max(p2 - p1, 1), 0.0)
        sec = max(t2 + per_pair * (full_pairs - p2), t2)
    return {
        "value": 1.0 / sec, "unit": "iters/s", "cores": cores, "kind": "oracle",
        "host_nproc": os.cpu_count(),
        "sample": (f"oracle walk at random supports per player, one iteration each: "
                   + ", ".join(f"{p} pairs {x:.3f} s" for p, x in pts)
                   + f"; extrapolated linearly in pairs from the last two to the full ranges' {full_pairs} pairs"),
    }


def he_params(shapes, seed):
    rng = np.random.default_rng(seed)
    return [((rng.standard_normal((o, i)) * np.sqrt(2.0 / i)).astype(np.float32), np.zeros(o, np.float32))
            for o, i in shapes]


def timed(solver, steps, warmup):
    import torch

    solver.iterate(warmup)
    solver.synchronize()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(solver.stream)
    solver.iterate(steps)
    ev1.record(solver.stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def tree_sweep(args, seed, steps, warmup):
    """Turn subgame to showdown: ms/iter and the backward kernel's HBM roofline."""
    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P

    spec, r = I.turn_config(seed)
    log(f"building turn subgame seed={seed} {spec}")
    tree = P.Tree(**spec)
    solver = P.Solver(tree, r, P.SolverConfig(dtype=args.dtype))
    esz = 8 if args.dtype == "f64" else 4
    alg_bytes = 4 * esz * tree.n_rows * tree.n_hands   # R and S, each read and written once
    ms = timed(solver, steps, warmup)
    visits = history_visits(tree, spec, r)
    pms, pl = solver.profile(args.profile_iters)
    pms, pl = pms / args.profile_iters, pl // args.profile_iters
    achieved = alg_bytes / (pms[3] * 1e-3) / 1e9
    expl, _ = solver.exploitability()
    traffic = MEASURED_TRAFFIC["turn_backward_iteration"] if seed == 0 and args.dtype == "f32" else None
    out = {
        "workload": f"turn subgame to showdown, seed {seed}",
        "board": spec["board"], "pot": spec["pot"], "stacks": list(spec["stacks"]),
        "nodes": tree.n_nodes, "decision_nodes": tree.n_decision, "chance_nodes": tree.n_chance,
        "action_rows": tree.n_rows, "hands": tree.n_hands, "levels": tree.n_levels,
        "state_bytes_R_S": 2 * esz * tree.n_rows * tree.n_hands_padded,
        "ms_per_iter": ms, "iters_per_s": 1000.0 / ms,
        "history_visits_per_iter": visits, "history_visits_per_s": visits * 1000.0 / ms,
        "iteration_hbm_frac": (alg_bytes / (ms * 1e-3) / 1e9) / HBM_PEAK_GBS,
        "kernel_ms_per_iter": {k: float(v) for k, v in zip(CLASSES, pms)},
        "exploitability_mbb_per_hand": expl * 100.0,
        "roofline": {
            "kernel": "k_backward<float,0> (values, DCFR regret and average-strategy update)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_note": "HBM bytes per iteration over all backward launches (hardware counters)",
            "counter_gbs": None if traffic is None else traffic / (pms[3] * 1e-3) / 1e9,
            "counter_frac": None if traffic is None else traffic / (pms[3] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "avg_launch_us": 1e3 * pms[3] / max(pl[3], 1), "launches_per_iter": int(pl[3]),
            "alg_bytes_per_iter": alg_bytes,
        },
    }
    log(f"turn: {ms:.4f} ms/iter, kernels {out['kernel_ms_per_iter']}")
    return out, spec, r


def batch_sweep(args, seed, steps, warmup, individual=True):
    """256 river/turn subgames of uneven size in one forest: ms per batched
    iteration (after the autotuner) against the same subgames solved one at a
    time, and the backward kernel's HBM roofline over the whole forest."""
    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P

    cases = I.batch_config(seed, lambda s: P.Tree(**s).n_nodes, n=256, river_share=0.7, lo=10, hi=2000)
    trees = [P.Tree(**s) for s, _ in cases]
    nodes = np.array([t.n_nodes for t in trees])
    rows = np.array([t.n_rows for t in trees])
    hands = np.array([t.n_hands for t in trees])
    n_river = sum(1 for s, _ in cases if len(s["board"]) == 5)
    log(f"batch of {len(trees)}: {n_river} river + {len(trees) - n_river} turn, nodes {nodes.min()}..{nodes.max()} "
        f"(median {int(np.median(nodes))}), {int(nodes.sum())} in all")
    b = P.Batch(trees, np.stack([r for _, r in cases]), P.SolverConfig(dtype=args.dtype))
    before, after = b.autotune(5)
    log(f"autotune: {before:.4f} -> {after:.4f} ms/iter")
    ms = timed(b, steps, warmup)
    pms, pl = b.profile(args.profile_iters)
    pms, pl = pms / args.profile_iters, pl // args.profile_iters
    esz = 8 if args.dtype == "f64" else 4
    alg_bytes = 4 * esz * float((rows * hands).sum())
    achieved = alg_bytes / (pms[3] * 1e-3) / 1e9
    expl, _ = b.exploitability_all()
    # the same forest with every iteration of the timed window in one
    # persistent cooperative launch (grid barriers between the phases);
    # identical iterates, so the same exploitability
    ms_persist = None
    if not args.no_persistent:
        pb = P.Batch(trees, np.stack([r for _, r in cases]), P.SolverConfig(dtype=args.dtype))
        pb.set_launch(True)
        ms_persist = timed(pb, steps, warmup)
        pb.close()
    log(f"batch: graph {ms:.4f} ms/iter, persistent launch {ms_persist} ms/iter")
    traffic = MEASURED_TRAFFIC["batch_backward_iteration"] if seed == 0 and args.dtype == "f32" else None
    out = {
        "workload": f"256 river/turn subgames in one forest, seed {seed}",
        "subgames": len(trees), "river": n_river, "turn": len(trees) - n_river,
        "nodes_min": int(nodes.min()), "nodes_median": int(np.median(nodes)), "nodes_max": int(nodes.max()),
        "nodes_total": int(nodes.sum()), "action_rows_total": int(rows.sum()),
        "ms_per_iter": ms, "iters_per_s": 1000.0 / ms,
        "persistent_launch_ms_per_iter": ms_persist,
        "persistent_launch_note": "all timed iterations in one cooperative launch of a resident grid, grid "
                                  "barriers between level sweeps and terminals; ms_per_iter is the autotuned "
                                  "graph of per-level launches",
        "autotune_ms_per_iter_before_after": [before, after],
        "kernel_ms_per_iter": {k: float(v) for k, v in zip(CLASSES, pms)},
        "exploitability_mbb_per_hand_mean": float(np.mean(expl)) * 100.0,
        "roofline": {
            "kernel": "k_backward<float,0> over the forest", "bound": "hbm", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_note": "HBM bytes per iteration over the backward launches of one tuned iteration (hardware "
                            "counters)",
            "counter_gbs": None if traffic is None else traffic / (pms[3] * 1e-3) / 1e9,
            "counter_frac": None if traffic is None else traffic / (pms[3] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "avg_launch_us": 1e3 * pms[3] / max(pl[3], 1), "launches_per_iter": int(pl[3]),
            "alg_bytes_per_iter": alg_bytes,
        },
    }
    b.close()
    if individual:
        # the same subgames one at a time, default launch schedule where no
        # size bucket was tuned; iterates are bitwise those of the batch
        tot = 0.0
        isteps = max(10, steps // 4)
        for (s, r), t in zip(cases, trees):
            one = P.Solver(t, r, P.SolverConfig(dtype=args.dtype))
            tot += timed(one, isteps, 3)
            one.close()
        out["one_at_a_time_ms_per_iter"] = tot
        out["batched_speedup"] = tot / ms
        log(f"batch: {ms:.4f} ms/iter batched, {tot:.4f} ms one at a time ({tot / ms:.1f}x)")
    return out


def suit_iso_sweep(args, steps, warmup):
    """Lossless suit isomorphism: the turn abstraction of the tree-sweep line
    on a one-suit board (the three other suits interchangeable) with
    suit-symmetric Dirichlet ranges, timed plain and with suit_iso = 1 (the
    iterates agree up to rounding order; tested)."""
    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P

    board = [50, 46, 26, 10]
    rng = np.random.default_rng(0)
    r = np.stack([I.symmetric_range(rng, board), I.symmetric_range(rng, board)])
    spec = dict(board=board, pot=100, stacks=(400, 400), sizes=[33, 75, 150], allin=True, max_raises=3,
                depth_limit=0)
    tree = P.Tree(**spec)
    out = {"workload": "turn to showdown on a one-suit board, suit-symmetric Dirichlet(1) ranges, seed 0",
           "board": board, "pot": spec["pot"], "stacks": list(spec["stacks"]), "nodes": tree.n_nodes}
    for name, iso in (("plain", 0), ("suit_iso", 1)):
        s = P.Solver(tree, r, P.SolverConfig(dtype=args.dtype, suit_iso=iso))
        out[f"swept_nodes_{name}"] = s.swept_nodes()
        out[f"ms_per_iter_{name}"] = timed(s, steps, warmup)
        s.close()
    out["speedup"] = out["ms_per_iter_plain"] / out["ms_per_iter_suit_iso"]
    log(f"suit isomorphism: {out['ms_per_iter_plain']:.4f} -> {out['ms_per_iter_suit_iso']:.4f} ms/iter "
        f"({out['swept_nodes_plain']} -> {out['swept_nodes_suit_iso']} swept nodes)")
    return out


def pruning_sweep(args, spec, r, steps, warmup, warm_iters=100, eps=0.1):
    """Online pruning on the turn of the tree-sweep line.  The bounds are the
    node values under the average strategies after a short solve, widened by
    eps times each hand's spread between sibling actions (standing in for the
    intervals of a value-network ensemble, which this library does not
    train); the dominance test runs on the GPU, the dominated actions leave
    the tree, and the reduced tree is timed against the full one."""
    import torch

    from paper_2605_19928_amd import pcfr as P

    tree = P.Tree(**spec)
    s = P.Solver(tree, r, P.SolverConfig(dtype=args.dtype))
    ms_full = timed(s, steps, warmup)
    s.iterate(warm_iters)
    t0 = time.perf_counter()
    V = s.node_values()
    s.close()
    e = tree.export()
    dec = np.flatnonzero(e["type"] == P.NODE_DECISION)
    cnt = e["n_child"][dec]
    par = np.repeat(dec, cnt)
    child = (np.repeat(e["first_child"][dec] - np.cumsum(cnt) + cnt, cnt) + np.arange(int(cnt.sum())))
    dev = V.device
    C = torch.from_numpy(child).to(dev)
    Pn = torch.from_numpy(par).to(dev)
    v = V[C, torch.from_numpy(e["player"][par].astype(np.int64)).to(dev)]
    del V
    n = tree.n_nodes
    idx = Pn[:, None].expand_as(v)
    vmax = torch.full((n, P.NCOMBO), -np.inf, dtype=torch.float64, device=dev).scatter_reduce(0, idx, v, "amax")
    vmin = torch.full((n, P.NCOMBO), np.inf, dtype=torch.float64, device=dev).scatter_reduce(0, idx, v, "amin")
    spread = (vmax - vmin)[Pn]
    del vmax, vmin
    lo = torch.full((n, P.NCOMBO), -np.inf, dtype=torch.float64, device=dev)
    hi = torch.full((n, P.NCOMBO), np.inf, dtype=torch.float64, device=dev)
    lo[C] = v - eps * spread
    hi[C] = v + eps * spread
    del v, spread
    t1 = time.perf_counter()
    flags = tree.prune_dominated(r, lo, hi)
    t2 = time.perf_counter()
    del lo, hi
    pruned, _ = tree.prune(flags)
    t3 = time.perf_counter()
    s2 = P.Solver(pruned, r, P.SolverConfig(dtype=args.dtype))
    ms_pruned = timed(s2, steps, warmup)
    s2.close()
    out = {
        "workload": "turn of the tree-sweep line; bounds = node values of the average strategies after "
                    f"{warmup + steps + warm_iters} iterations +- {eps} x the per-hand spread of sibling actions",
        "bounds_kind": "heuristic: point values of a short solve widened by a margin, not sound bounds (the "
                       "value-network ensemble that gives sound ones is not part of this library); the line "
                       "times the dominance test and the reduced tree, not a lossless pruning",
        "nodes_full": n, "nodes_pruned": pruned.n_nodes, "rho": pruned.n_nodes / n,
        "actions_removed": int(flags.sum()), "action_rows_full": tree.n_rows, "action_rows_pruned": pruned.n_rows,
        "bounds_ms": 1e3 * (t1 - t0), "dominance_test_ms": 1e3 * (t2 - t1), "tree_reduction_ms": 1e3 * (t3 - t2),
        "ms_per_iter_full": ms_full, "ms_per_iter_pruned": ms_pruned, "speedup": ms_full / ms_pruned,
    }
    log(f"pruning: {n} -> {pruned.n_nodes} nodes (rho {out['rho']:.3f}), {ms_full:.4f} -> {ms_pruned:.4f} ms/iter, "
        f"dominance test {out['dominance_test_ms']:.1f} ms")
    return out


def rbp_sweep(args, spec, r, steps, warmup, warm_iters=100):
    """Regret-based pruning of unreachable subtrees (exact: the iterates equal
    the unpruned ones) without and with dynamic thresholding (actions below
    thr0 / sqrt(t) dropped): ms/iter pruned vs unpruned at the same threshold
    after warm_iters iterations, the nodes skipped in the last iteration, and
    the exploitability after the same number of iterations.  Two range
    profiles: the turn of the tree-sweep line with full Dirichlet ranges
    (every action is some hand's choice, so little is unreachable), and a
    turn whose players hold 64 combos each."""
    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P

    out = []
    sspec, sr = I.turn_config(0, support=64)
    for label, sp, rr in (("full Dirichlet(1) ranges", spec, r), ("64-combo supports", sspec, sr)):
        tree = P.Tree(**sp)
        for thr in (0.0, 0.05):
            res = {"ranges": label, "threshold_thr0": thr, "nodes": tree.n_nodes}
            for prune in (0, 1):
                s = P.Solver(tree, rr, P.SolverConfig(dtype=args.dtype, threshold=thr, prune=prune))
                s.iterate(warm_iters)
                ms = timed(s, steps, warmup)
                res["ms_per_iter_pruned" if prune else "ms_per_iter_unpruned"] = ms
                if prune:
                    res["nodes_skipped_last_iter"] = s.unreached_nodes()
                    res["iterations"] = warm_iters + warmup + steps
                    e, _ = s.exploitability()
                    res["exploitability_mbb_per_hand"] = e * 100.0
                s.close()
            res["skipped_share"] = res["nodes_skipped_last_iter"] / tree.n_nodes
            res["speedup"] = res["ms_per_iter_unpruned"] / res["ms_per_iter_pruned"]
            log(f"regret-based pruning, {label}, thr0={thr}: {res['ms_per_iter_unpruned']:.4f} -> "
                f"{res['ms_per_iter_pruned']:.4f} ms/iter, {res['nodes_skipped_last_iter']} of {tree.n_nodes} nodes "
                f"skipped, exploitability {res['exploitability_mbb_per_hand']:.1f} mbb/hand")
            out.append(res)
    return out


def learned_leaf_sweep(args, n_train=4096, gen_iters=200, train_steps=2000, iters=300):
    """The learned leaf against the exact solve, trained in the bench run
    (seeded, so every run regenerates the same network): n_train random turn
    subgames solved by the batched plain solver give the training samples,
    the library's bf16 kernels train the 4 x 1536 network with Adam, and the
    headline flop is solved `iters` iterations with that network at its
    depth-limit leaves and, exactly, dealt out to showdown.  Matched quality:
    the root values under the average strategies of the learned-leaf solve
    are within `root_value_gap` of the exact solve's after `iters`
    iterations; the exact solver's own root values reach that distance from
    its final values only after `exact_iterations_to_match` iterations, and
    the time for that is set against the learned-leaf solve's."""
    import torch

    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P
    from paper_2605_19928_amd import train as T

    t0 = time.perf_counter()
    X, Y, M, _ = T.generate(seed=101, n=n_train, iters=gen_iters, batch=512, dtype="f32")
    gen_s = time.perf_counter() - t0
    net = P.LeafNet(P.LEAF_D_IN, 1536, 4, P.LEAF_D_OUT, max_batch=1088)
    net.set_params(he_params(net.layer_shapes(), 0))
    t0 = time.perf_counter()
    hist = T.train(net, X, Y, M, steps=train_steps, batch=1024, lr=5e-4, log_every=max(train_steps // 4, 1))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del X, Y, M
    spec, r = I.flop_config(args.seed)
    tree = P.Tree(**spec)
    dl = P.Solver(tree, r, P.SolverConfig(dtype=args.dtype))
    dl.attach_leafnet(net)
    dl.autotune(3)
    ms_dl = timed(dl, iters, 0)
    v_dl = dl.root_cfv("avg")
    e_dl, _ = dl.exploitability()
    dl.close()
    stub = P.Solver(tree, r, P.SolverConfig(dtype=args.dtype))
    stub.iterate(iters)
    v_stub = stub.root_cfv("avg")
    stub.close()
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    tx = P.Tree(**dict(spec, depth_limit=0))
    build_s = time.perf_counter() - t0
    ex = P.Solver(tx, r, P.SolverConfig(dtype=args.dtype))
    checkpoints = [k for k in (1, 2, 4, 8, 16, 32, 64, 128, 256) if k < iters] + [iters]
    snaps, done, ms_ex = {}, 0, 0.0
    for k in checkpoints:
        ms_ex += timed(ex, k - done, 0) * (k - done)
        done = k
        snaps[k] = ex.root_cfv("avg")
    e_ex, _ = ex.exploitability()
    # one more iteration with per-launch timing: the sweep's kernel split and
    # its algorithmic HBM fractions (R and S read and written once per
    # action row and hand, as for the turn line)
    esz = 8 if args.dtype == "f64" else 4
    alg_ex = 4 * esz * tx.n_rows * tx.n_hands
    pms_ex, _ = ex.profile(1)
    ex.close()
    del ex
    torch.cuda.empty_cache()
    ms_ex /= iters
    ref = snaps[iters]
    gap = lambda v: float((r * np.abs(v - ref)).sum() / (2.0 * pair_mass(r)) * 100.0)
    g_dl, g_stub = gap(v_dl), gap(v_stub)
    curve = [(k, gap(snaps[k])) for k in checkpoints[:-1]]
    match = next((k for k, g in curve if g <= g_dl), iters)
    out = {
        "workload": f"the headline flop (seed {args.seed}); network trained in this run on {n_train} turn subgames "
                    f"x {gen_iters} solver iterations, {train_steps} Adam steps (batch 1024)",
        "generate_s": gen_s, "train_s": train_s, "train_loss_first_last": [hist[0][1], hist[-1][1]],
        "iterations": iters,
        "learned_leaf_ms_per_iter": ms_dl, "learned_leaf_iters_per_s": 1000.0 / ms_dl,
        "learned_leaf_exploitability_mbb_per_hand_in_depth_limited_game": e_dl * 100.0,
        "exact_nodes": tx.n_nodes, "exact_tree_build_s": build_s,
        "exact_ms_per_iter": ms_ex, "exact_iters_per_s": 1000.0 / ms_ex,
        "exact_exploitability_mbb_per_hand": e_ex * 100.0,
        "exact_state_bytes_R_S": 2 * esz * tx.n_rows * tx.n_hands_padded,
        "exact_kernel_ms_per_iter": {k: float(v) for k, v in zip(CLASSES, pms_ex)},
        "exact_backward_alg_hbm_frac": alg_ex / (float(pms_ex[3]) * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "exact_iteration_alg_hbm_frac": alg_ex / (ms_ex * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "root_value_gap_mbb_per_hand": {"learned_leaves_vs_exact": g_dl, "checkdown_equity_leaves_vs_exact": g_stub},
        "exact_root_value_gap_by_iterations": curve,
        "exact_iterations_to_match": match,
        "time_to_matched_quality_ms": {"learned_leaf": ms_dl * iters, "exact": ms_ex * match},
        "speedup_at_matched_quality": (ms_ex * match) / (ms_dl * iters),
    }
    log(f"learned leaf: {ms_dl:.4f} ms/iter, gap {g_dl:.1f} mbb/hand to exact ({ms_ex:.2f} ms/iter); exact needs "
        f"{match} iterations for that gap: {out['speedup_at_matched_quality']:.1f}x")
    log(f"exact flop: {tx.n_nodes} nodes, {out['exact_state_bytes_R_S'] / 1e9:.1f} GB of R + S, backward "
        f"{out['exact_backward_alg_hbm_frac']:.3f} and iteration {out['exact_iteration_alg_hbm_frac']:.3f} of HBM peak "
        f"(algorithmic)")
    return out


def pair_mass(r):
    """Joint mass of compatible hand pairs."""
    from paper_2605_19928_amd import inputs as I

    cc = I.combo_cards()
    card = np.zeros(52)
    np.add.at(card, cc[:, 0], r[1])
    np.add.at(card, cc[:, 1], r[1])
    comp = r[1].sum() - card[cc[:, 0]] - card[cc[:, 1]] + r[1]
    return float((r[0] * comp).sum())


def spr_sweep(args, steps, warmup, seed=0):
    """The turn abstraction at stack-to-pot ratios 1, 2, 4 and 8: nodes, sum of
    A*H over decision nodes, R + S bytes, ms/iter and the backward kernels'
    algorithmic HBM fraction (16 B per (row, hand) in FP32); only trees whose
    R + S exceed the 256 MB last-level cache count toward a bandwidth claim."""
    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P

    out = []
    esz = 8 if args.dtype == "f64" else 4
    for spr in (1, 2, 4, 8):
        spec, r = I.turn_config(seed, spr=spr)
        tree = P.Tree(**spec)
        s = P.Solver(tree, r, P.SolverConfig(dtype=args.dtype))
        ms = timed(s, steps, warmup)
        pms, _ = s.profile(args.profile_iters)
        pms = pms / args.profile_iters
        sum_ah = tree.n_rows * tree.n_hands
        alg = 4 * esz * sum_ah
        out.append({"spr": spr, "pot": spec["pot"], "stacks": list(spec["stacks"]), "nodes": tree.n_nodes,
                    "decision_nodes": tree.n_decision, "chance_nodes": tree.n_chance, "sum_AH": sum_ah,
                    "r_plus_s_bytes": 2 * esz * sum_ah, "ms_per_iter": ms,
                    "backward_ms_per_iter": float(pms[3]),
                    "backward_alg_hbm_frac": alg / (pms[3] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "iteration_alg_hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "counts_toward_bandwidth_claim": 2 * esz * sum_ah > 256 * (1 << 20)})
        s.close()
        log(f"turn SPR {spr}: {tree.n_nodes} nodes, {ms:.4f} ms/iter, backward "
            f"{out[-1]['backward_alg_hbm_frac']:.3f} of HBM peak (algorithmic)")
    return out


def flop_batch_sweep(args, steps, warmup, sizes=(8, 32)):
    """B depth-limited flops (the headline abstraction, each with its own
    board and ranges) in one forest with one leaf network, so each iteration
    sends B x leaves x next cards rows through the same GEMMs: ms per batched
    iteration, per flop, and the hidden-layer GEMM rate at that many rows."""
    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P

    out = []
    for B in sizes:
        cases = [I.flop_config(args.seed + k) for k in range(B)]
        trees = [P.Tree(**s) for s, _ in cases]
        b = P.Batch(trees, np.stack([r for _, r in cases]), P.SolverConfig(dtype=args.dtype))
        n_leaves, n_next = b.leaf_rows()
        rows = n_leaves * n_next
        net = P.LeafNet(P.LEAF_D_IN, 1536, 4, P.LEAF_D_OUT, max_batch=rows)
        net.set_params(he_params(net.layer_shapes(), 7))
        b.attach_leafnet(net)
        before, after = b.autotune(5)
        ms = timed(b, steps, warmup)
        pms, pl = b.profile(args.profile_iters)
        pms, pl = pms / args.profile_iters, pl // args.profile_iters
        shapes = net.layer_shapes()
        hidden_flops = 2.0 * rows * sum(o * i for o, i in shapes[:-1])
        all_flops = 2.0 * rows * sum(o * i for o, i in shapes)
        expl, _ = b.exploitability_all()
        out.append({
            "workload": f"{B} depth-limited flops (seeds {args.seed}..{args.seed + B - 1}) in one forest, "
                        f"leaf network 1536x4",
            "subgames": B, "nodes_total": int(sum(t.n_nodes for t in trees)), "network_rows": rows,
            "ms_per_iter": ms, "ms_per_flop_iter": ms / B, "flop_iters_per_s": 1000.0 * B / ms,
            "autotune_ms_per_iter_before_after": [before, after], "leaf_gemm_tiles": net.tiles,
            "kernel_ms_per_iter": {k: float(v) for k, v in zip(CLASSES, pms)},
            "leaf_gemm_hidden_tflops": hidden_flops / (pms[5] * 1e-3) / 1e12,
            "leaf_gemm_all_layers_tflops": all_flops / ((pms[5] + pms[6]) * 1e-3) / 1e12,
            "exploitability_mbb_per_hand_mean": float(np.mean(expl)) * 100.0,
        })
        log(f"{B} flops batched: {ms:.4f} ms/iter ({ms / B:.4f} ms per flop), {rows} network rows, hidden GEMM "
            f"{out[-1]['leaf_gemm_hidden_tflops']:.0f} TFLOP/s")
        b.close()
        net.close()
    return out


def preflop_sweep(args, steps, warmup):
    """Preflop root (no board, pot 20, 100 bb behind, {50, 100}% with up to 3
    bets/raises, no all-in) solved over the 169 hand classes, its leaves at the
    flop deal valued by the flop-level network (2705 -> 4 x 1536 -> 2652, He
    init) on the 1755 canonical flops: ms per iteration and the GEMM rate at
    that many rows.  The paper's preflop street takes 3.48 ms per iteration
    (Table 2; its own tree and CPU/GPU split), context only."""
    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P

    spec, r = I.preflop_config(args.seed)
    tree = P.Tree(**spec)
    s = P.Solver(tree, r, P.SolverConfig(dtype=args.dtype))
    n_leaves, n_next = s.leaf_rows()
    rows = n_leaves * n_next
    net = P.LeafNet(P.LEAF_D_IN, 1536, 4, P.LEAF_D_OUT, max_batch=rows)
    net.set_params(he_params(net.layer_shapes(), 7))
    s.attach_leafnet(net)
    before, after = s.autotune(3)
    ms = timed(s, steps, warmup)
    pms, pl = s.profile(args.profile_iters)
    pms, pl = pms / args.profile_iters, pl // args.profile_iters
    shapes = net.layer_shapes()
    hidden_flops = 2.0 * rows * sum(o * i for o, i in shapes[:-1])
    all_flops = 2.0 * rows * sum(o * i for o, i in shapes)
    expl, _ = s.exploitability()
    out = {
        "workload": f"preflop root, seed {args.seed}: {tree.n_nodes} nodes, {n_leaves} leaves at the flop deal x "
                    f"{n_next} canonical flops, 169 hand classes, leaf network 1536x4",
        "spec": {k: (list(v) if isinstance(v, tuple) else v) for k, v in spec.items()},
        "nodes": tree.n_nodes, "leaves": n_leaves, "canonical_flops": n_next, "network_rows": rows,
        "hands": tree.n_hands, "ms_per_iter": ms, "iters_per_s": 1000.0 / ms,
        "autotune_ms_per_iter_before_after": [before, after], "leaf_gemm_tiles": net.tiles,
        "kernel_ms_per_iter": {k: float(v) for k, v in zip(CLASSES, pms)},
        "leaf_gemm_hidden_tflops": hidden_flops / (pms[5] * 1e-3) / 1e12,
        "leaf_gemm_all_layers_tflops": all_flops / ((pms[5] + pms[6]) * 1e-3) / 1e12,
        "leaf_flops_per_iter": all_flops,
        "exploitability_mbb_per_hand": expl * 100.0,
        "paper_preflop_ms_per_iter": 3.48,
        "paper_note": "Table 2, preflop street, 5 CPU threads + GPU leaf evaluation on another machine and tree",
    }
    log(f"preflop: {ms:.4f} ms/iter, {rows} network rows, hidden GEMM {out['leaf_gemm_hidden_tflops']:.0f} TFLOP/s")
    s.close()
    net.close()
    return out


def flop_2000_rows(args, steps, warmup):
    """A full iteration of a depth-limited flop with about 2,000 network rows:
    three bet sizes (33, 66, 100% of the pot) and three raises give 43
    network leaves x 49 turn cards = 2,107 rows (the headline's two sizes give
    21 leaves, 1,029 rows, beside 14 all-in leaves valued by exact equity)."""
    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P

    spec, r = I.flop_config(args.seed, sizes=(33, 66, 100), max_raises=3)
    tree = P.Tree(**spec)
    s = P.Solver(tree, r, P.SolverConfig(dtype=args.dtype))
    n_leaves, n_next = s.leaf_rows()
    rows = n_leaves * n_next
    net = P.LeafNet(P.LEAF_D_IN, 1536, 4, P.LEAF_D_OUT, max_batch=rows)
    net.set_params(he_params(net.layer_shapes(), 7))
    s.attach_leafnet(net)
    before, after = s.autotune(3)
    ms = timed(s, steps, warmup)
    pms, pl = s.profile(args.profile_iters)
    pms, pl = pms / args.profile_iters, pl // args.profile_iters
    shapes = net.layer_shapes()
    hidden_flops = 2.0 * rows * sum(o * i for o, i in shapes[:-1])
    n_hidden = max(int(pl[5]), 1)
    hidden_tflops = hidden_flops / (pms[5] * 1e-3) / 1e12
    out = {
        "workload": f"depth-limited flop, seed {args.seed}, bet sizes 33/66/100% + all-in, 3 raises",
        "nodes": tree.n_nodes, "network_leaves": n_leaves, "allin_leaves": tree.n_allin, "network_rows": rows,
        "ms_per_iter": ms, "iters_per_s": 1000.0 / ms, "autotune_ms_per_iter_before_after": [before, after],
        "leaf_gemm_tiles": list(net.tiles), "kernel_ms_per_iter": {k: float(v) for k, v in zip(CLASSES, pms)},
        "leaf_gemm_hidden_tflops": hidden_tflops, "leaf_gemm_hidden_frac": hidden_tflops / BF16_PEAK_TFLOPS,
        "leaf_gemm_hidden_avg_launch_us": 1e3 * pms[5] / n_hidden,
    }
    s.close()
    net.close()
    log(f"flop with {rows} network rows: {ms:.4f} ms/iter, hidden GEMM {hidden_tflops:.0f} TFLOP/s "
        f"({out['leaf_gemm_hidden_frac']:.3f} of peak)")
    return out


def gemm_shape_point(args, m=2048, reps=50):
    """The leaf network's forward at m rows (the second GEMM shape point),
    after the tile autotuner: us per forward and TFLOP/s."""
    import torch

    from paper_2605_19928_amd import pcfr as P
    from paper_2605_19928_amd import train as T

    net = P.LeafNet(P.LEAF_D_IN, 1536, 4, P.LEAF_D_OUT, max_batch=m)
    net.set_params(he_params(net.layer_shapes(), 0))
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.standard_normal((m, P.LEAF_D_IN)).astype(np.float32)).cuda()
    net.autotune(m, 10)
    ms = T.forward_ms(net, x, reps=reps)
    flops = 2.0 * m * sum(o * i for o, i in net.layer_shapes())
    out = {"rows": m, "us_per_forward": ms * 1e3, "tflops": flops / (ms * 1e-3) / 1e12, "tiles": list(net.tiles)}
    net.close()
    log(f"leaf network forward at {m} rows: {ms * 1e3:.1f} us, {out['tflops']:.0f} TFLOP/s")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    from paper_2605_19928_amd import inputs as I
    from paper_2605_19928_amd import pcfr as P

    if args.calibrate_mb:
        import torch

        x = torch.ones(args.calibrate_mb * (1 << 18), dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        log(f"calibration kernel: read {args.calibrate_mb} MiB, wrote {args.calibrate_mb} MiB")
        del x, y

    if args.workload == "batch":
        out = batch_sweep(args, args.seed, args.steps, args.warmup, individual=not args.no_one_at_a_time)
        result = {
            "metric": "DCFR ms/iter & iters/sec, flop depth-limited subgame; exploitability mbb/hand",
            "value": out["iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": out["ms_per_iter"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
            "config": {k: v for k, v in out.items() if k not in ("roofline", "kernel_ms_per_iter")},
            "roofline": out["roofline"],
        }
        print(json.dumps(result), flush=True)
        return

    if args.workload == "flop-batch":
        out = flop_batch_sweep(args, args.steps, args.warmup, sizes=(args.batch_flops,))[0]
        result = {
            "metric": "DCFR ms/iter & iters/sec, flop depth-limited subgame; exploitability mbb/hand",
            "value": out["flop_iters_per_s"], "unit": "flop iters/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": out["ms_per_iter"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
            "config": {k: v for k, v in out.items() if k != "kernel_ms_per_iter"},
            "kernel_ms_per_iter": out["kernel_ms_per_iter"],
        }
        print(json.dumps(result), flush=True)
        return

    if args.workload == "datagen":
        # training data for the leaf network at the recipe's solve depth: random
        # turn subgames solved by the batched plain solver, root targets sampled
        from paper_2605_19928_amd import train as T

        n, iters, batch = args.datagen_subgames, args.datagen_iters, 512
        t0 = time.perf_counter()
        X, Y, M, specs = T.generate(seed=args.seed + 1000, n=n, iters=iters, batch=batch, dtype=args.dtype, log=log)
        import torch

        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        nodes = [P.Tree(**s).n_nodes for s, _ in specs[:256]]
        rate = n / wall
        result = {
            "metric": "leaf-network training data: turn subgames solved per second",
            "value": rate, "unit": "subgames/s", "n_gpus": 1, "steps": iters, "warmup": 0,
            "ms_per_step": 1e3 * wall / iters, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": args.dtype, "data": "synthetic",
            "config": {"workload": f"{n} random turn subgames (Dirichlet(0.5-2) ranges, log-uniform pot and SPR "
                                   f"0.1-8, 75% + all-in, 2 raises) x {iters} DCFR iterations, batches of {batch}",
                       "subgames": n, "iterations": iters, "batch": batch,
                       "nodes_per_subgame_median": float(np.median(nodes)),
                       "wall_s": wall, "subgame_iterations_per_s": n * iters / wall,
                       "extrapolated_s_for_100k_subgames": 1e5 / rate},
        }
        log(f"datagen: {n} subgames x {iters} iterations in {wall:.1f} s ({rate:.1f} subgames/s; "
            f"100k would take {1e5 / rate / 60:.1f} min)")
        print(json.dumps(result), flush=True)
        return

    if args.workload == "preflop":
        out = preflop_sweep(args, args.steps, args.warmup)
        result = {
            "metric": "DCFR ms/iter & iters/sec, preflop root with leaves at the flop deal; exploitability mbb/hand",
            "value": out["iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": out["ms_per_iter"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
            "config": {k: v for k, v in out.items() if k != "kernel_ms_per_iter"},
            "kernel_ms_per_iter": out["kernel_ms_per_iter"],
        }
        print(json.dumps(result), flush=True)
        return

    if args.workload == "turn":
        sweep, spec, r = tree_sweep(args, args.seed, args.steps, args.warmup)
        result = {
            "metric": "DCFR ms/iter & iters/sec, flop depth-limited subgame; exploitability mbb/hand",
            "value": sweep["iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": sweep["ms_per_iter"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
            "config": {k: v for k, v in sweep.items() if k not in ("roofline", "kernel_ms_per_iter")},
            "roofline": sweep["roofline"],
        }
        if not args.no_cpu_baseline:
            log("timing the CPU oracle on a bounded sample")
            result["cpu_baseline"] = cpu_baseline(spec, r, args.cpu_seconds)
        print(json.dumps(result), flush=True)
        return

    spec, r = I.flop_config(args.seed)
    log(f"building depth-limited flop subgame seed={args.seed} {spec}")
    tree = P.Tree(**spec)
    solver = P.Solver(tree, r, P.SolverConfig(dtype=args.dtype))
    n_leaves, n_next = solver.leaf_rows()
    rows = n_leaves * n_next
    net = P.LeafNet(P.LEAF_D_IN, 1536, 4, P.LEAF_D_OUT, max_batch=rows)
    params = he_params(net.layer_shapes(), 7)
    net.set_params(params)
    solver.attach_leafnet(net)
    flops_alg = 2.0 * rows * sum(o * i for o, i in net.layer_shapes())
    tune_before, tune_after = solver.autotune(5)
    log(f"autotune: {tune_before:.4f} -> {tune_after:.4f} ms/iter; network GEMM tiles {net.tiles}")
    ms = timed(solver, args.steps, args.warmup)
    log(f"{args.steps} steps: {ms:.4f} ms/iter")
    pms, pl = solver.profile(args.profile_iters)
    pms, pl = pms / args.profile_iters, pl // args.profile_iters
    # the dominant kernel: the hidden-layer GEMM instantiation (bias + ReLU,
    # bf16 out), launched once per hidden layer
    shapes = net.layer_shapes()
    hidden_flops = 2.0 * rows * sum(o * i for o, i in shapes[:-1])
    gemm_ms = pms[5]
    n_hidden = max(int(pl[5]), 1)
    achieved = (hidden_flops / n_hidden) / (gemm_ms / n_hidden * 1e-3) / 1e12
    all_gemm_tflops = flops_alg / ((pms[5] + pms[6]) * 1e-3) / 1e12
    gemm_traffic = None
    by_tile = MEASURED_TRAFFIC["gemm_hidden_by_tile"]
    if args.dtype == "f32" and all(t in by_tile for t in net.tiles[:-1]):
        gemm_traffic = float(np.mean([sum(by_tile[t]) for t in net.tiles[:-1]]))
    expl, _ = solver.exploitability()
    # the same K-step window five more times (after the exploitability, which
    # is then that of the timed run): the spread of the measurement
    repeats = [timed(solver, args.steps, 0) for _ in range(5)]
    log(f"kernel ms/iter {dict(zip(CLASSES, np.round(pms[:7], 4)))} launches {pl[:7].tolist()}")
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
            "workload": f"depth-limited flop subgame with leaf network, seed {args.seed}",
            "board": spec["board"], "pot": spec["pot"], "stacks": list(spec["stacks"]),
            "bet_sizes_pct": spec["sizes"], "allin": True, "max_raises_per_street": spec["max_raises"],
            "nodes": tree.n_nodes, "decision_nodes": tree.n_decision, "network_leaves": n_leaves,
            "allin_leaves": tree.n_allin, "next_cards": n_next, "network_rows": rows, "hands": tree.n_hands,
            "leaf_network": "2705 -> 4 x 1536 -> 2652 ReLU MLP, bf16 weights, fp32 accumulate, He init "
                            "(random weights: a throughput measurement; learned_leaf trains one and compares "
                            "against the exact solve)",
            "leaf_network_params": net.n_params,
            "leaf_flops_per_iter": flops_alg,
        },
        "exploitability_mbb_per_hand": expl * 100.0,
        "exploitability_note": "of the average strategy within the depth-limited game, leaves valued by the network",
        "repeat_ms_per_step": repeats,
        "repeat_note": "five more windows of the same K steps after the timed one (median "
                       f"{float(np.median(repeats)):.4f} ms, spread {100 * (max(repeats) - min(repeats)) / float(np.median(repeats)):.1f}%)",
        "history_visits_per_s": history_visits(tree, spec, r) * 1000.0 / ms,
        "history_visits_note": "per iteration, over every node, hand pairs with mass on both sides that share no "
                               "card with each other or the node's board; the paper reports about 2.0e10/s",
        "autotune_ms_per_iter_before_after": [tune_before, tune_after],
        "leaf_gemm_tiles": net.tiles,
        "kernel_ms_per_iter": {k: float(v) for k, v in zip(CLASSES, pms)},
        "leaf_gemm_all_layers_tflops": all_gemm_tflops,
        "roofline": {
            "kernel": "k_gemm_nt<BM,BN,1> (leaf network hidden layers: bias + ReLU, bf16 MFMA 32x32x16; "
                      "tile per layer from the autotuner)",
            "bound": "mfma",
            "achieved": achieved,
            "peak": BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / BF16_PEAK_TFLOPS,
            "traffic": gemm_traffic,
            "traffic_note": "HBM bytes per launch (hardware counters per tile variant, mean over the hidden "
                            "layers' tiles); algorithmic operand bytes are ~9.6 MB",
            "avg_launch_us": 1e3 * gemm_ms / n_hidden,
            "launches_per_iter": n_hidden,
            "alg_flops_per_launch": hidden_flops / n_hidden,
        },
    }
    del solver, net
    if not args.no_secondary:
        sweep, tspec, tr = tree_sweep(args, 0, max(20, args.steps // 4), 5)
        result["tree_sweep"] = sweep
        result["batch"] = batch_sweep(args, 0, max(20, args.steps // 4), 5)
        result["suit_isomorphism"] = suit_iso_sweep(args, max(20, args.steps // 4), 5)
        result["pruning"] = [pruning_sweep(args, tspec, tr, max(20, args.steps // 4), 5, eps=e) for e in (0.0, 0.05)]
        result["regret_based_pruning"] = rbp_sweep(args, tspec, tr, max(20, args.steps // 4), 5)
        result["turn_spr_sweep"] = spr_sweep(args, max(20, args.steps // 4), 5)
        result["leaf_gemm_m2048"] = gemm_shape_point(args)
        result["flop_2000_rows"] = flop_2000_rows(args, max(20, args.steps // 4), 5)
        result["flop_batch"] = flop_batch_sweep(args, max(20, args.steps // 4), 5)
        result["preflop"] = preflop_sweep(args, max(20, args.steps // 4), 5)
        result["hbm_copy_ceiling_gbs"] = copy_ceiling_gbs()
        if not args.no_learned:
            result["learned_leaf"] = learned_leaf_sweep(args)
        log(f"HBM copy ceiling: {result['hbm_copy_ceiling_gbs']:.0f} GB/s")
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(spec, r, args.cpu_seconds, leaf_params=params)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
