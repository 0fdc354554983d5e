"""Leaf-network study: train the depth-limit value network on subgames the
solver generates, then measure what it gains.

    python -m paper_2605_19928_amd.leafnet_study --out result.json

1. Data: ``--train`` random turn subgames (``inputs.leaf_training_config``:
   Dirichlet(0.5-2) ranges, log-uniform pot and stack-to-pot ratio; bet
   abstraction ``--train-sizes`` + all-in, ``--train-cap`` bets per street)
   solved ``--iters`` iterations each by the batched GPU solver; each gives
   one sample (normalised ranges, board, ratio -> values
   under the average strategies per pot and compatible opponent mass).  A
   disjoint held-out set (``--heldout``, another seed) is made the same way.
2. Training: the library's bf16-MFMA forward/backward/Adam kernels on the
   Huber loss, batch ``--batch``, cosine learning rate, suit-permutation
   augmentation.
3. Held-out error in mbb/hand (bb = 10 chips; hands weighted by own reach and
   compatible opponent mass), against the best constant predictor.
4. Gain over the method without the network: the plain solver run on the
   held-out subgames for k iterations; its error at the network's own
   evaluation time, and the iterations (and device time) it needs to match
   the network's error.
5. Flop comparison (``--flop``): the depth-limited flop subgame of the
   benchmark solved with the trained network at its leaves, against the same
   flop subgame solved exactly to showdown (turn and river dealt out, 5.1M
   nodes, ~120 GB of device memory): root values under the average
   strategies, their difference in mbb/hand, and ms per iteration of both.

Writes one JSON object to ``--out`` (and prints it).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs as I
from . import pcfr as P
from . import train as T


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def he_init(net: "P.LeafNet", seed: int):
    rng = np.random.default_rng(seed)
    return [((rng.standard_normal((o, i)) * np.sqrt(2.0 / i)).astype(np.float32), np.zeros(o, np.float32))
            for o, i in net.layer_shapes()]


def pair_mass(r):
    """Joint mass of compatible hand pairs, sum_h r0(h) * M_1(h)."""
    cc = I.combo_cards()
    card = np.zeros(52)
    np.add.at(card, cc[:, 0], r[1])
    np.add.at(card, cc[:, 1], r[1])
    comp = r[1].sum() - card[cc[:, 0]] - card[cc[:, 1]] + r[1]
    return float((r[0] * comp).sum())


def root_value_gap_mbb(v, w, r):
    """sum_i sum_h r_i(h) |v_i(h) - w_i(h)| / (2 Z) in mbb/hand (values in chips, bb = 10 chips)."""
    return float((r * np.abs(v - w)).sum() / (2.0 * pair_mass(r)) * 100.0)


def flop_comparison(net, seed: int, iters: int, out: dict):
    import torch

    spec, r = I.flop_config(seed)
    # depth-limited, network leaves
    tree = P.Tree(**spec)
    dl_runs = {}
    for zs in (True, False):
        dl = P.Solver(tree, r)
        n_leaves, n_next = dl.leaf_rows()
        dl.attach_leafnet(net)
        dl.set_leaf_zero_sum(zs)
        t_dl = T._elapsed_ms(lambda: dl.iterate(iters), dl.stream) / iters
        e_dl, _ = dl.exploitability()
        dl_runs[zs] = (t_dl, dl.root_cfv("avg"), e_dl)
        dl.close()
    # the same subgame with every leaf valued by check-down equity (no network)
    stub = P.Solver(tree, r)
    stub.iterate(iters)
    v_stub = stub.root_cfv("avg")
    stub.close()
    torch.cuda.empty_cache()
    # exact: dealt out to showdown
    full = dict(spec, depth_limit=0)
    t0 = time.perf_counter()
    tx = P.Tree(**full)
    log(f"flop to showdown: {tx.n_nodes} nodes, {tx.n_rows} action rows ({time.perf_counter() - t0:.1f} s to build)")
    ex = P.Solver(tx, r)
    log(f"flop to showdown: workspace {ex.workspace_bytes / 1e9:.1f} GB")
    ex.iterate(1)
    ex.synchronize()
    t_ex = T._elapsed_ms(lambda: ex.iterate(iters - 1), ex.stream) / max(iters - 1, 1)
    v_ex = ex.root_cfv("avg")
    e_ex, _ = ex.exploitability()
    ex.close()
    del ex
    torch.cuda.empty_cache()
    t_dl = dl_runs[True][0]
    out["flop"] = {
        "spec": {k: (list(v) if isinstance(v, tuple) else v) for k, v in spec.items()},
        "iterations": iters,
        "depth_limited": {"network_rows_per_iter": n_leaves * n_next, "ms_per_iter": t_dl,
                          "exploitability_mbb_per_hand_within_depth_limited_game":
                              {"zero_sum_leaves": dl_runs[True][2] * 100.0, "raw_leaves": dl_runs[False][2] * 100.0}},
        "exact_to_showdown": {"nodes": tx.n_nodes, "action_rows": tx.n_rows, "ms_per_iter": t_ex,
                              "exploitability_mbb_per_hand": e_ex * 100.0},
        "speedup_per_iteration": t_ex / t_dl,
        "root_value_gap_mbb_per_hand": {
            "trained_network_leaves_zero_sum_vs_exact": root_value_gap_mbb(dl_runs[True][1], v_ex, r),
            "trained_network_leaves_raw_vs_exact": root_value_gap_mbb(dl_runs[False][1], v_ex, r),
            "checkdown_equity_leaves_vs_exact": root_value_gap_mbb(v_stub, v_ex, r),
        },
    }
    log(json.dumps(out["flop"]))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train", type=int, default=16384)
    ap.add_argument("--heldout", type=int, default=512)
    ap.add_argument("--iters", type=int, default=400)
    ap.add_argument("--gen-batch", type=int, default=512)
    ap.add_argument("--width", type=int, default=1536)
    ap.add_argument("--depth", type=int, default=4)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--train-sizes", default="75", help="bet sizes (%% of pot) of the training subgames")
    ap.add_argument("--train-cap", type=int, default=2, help="bets/raises per street in the training subgames")
    ap.add_argument("--flop", action="store_true")
    ap.add_argument("--flop-iters", type=int, default=300)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    import torch

    res = {"train_subgames": args.train, "heldout_subgames": args.heldout, "solver_iterations": args.iters,
           "network": f"{P.LEAF_D_IN} -> {args.depth} x {args.width} -> {P.LEAF_D_OUT} ReLU, bf16 MFMA",
           "steps": args.steps, "batch": args.batch, "lr": args.lr}
    t0 = time.perf_counter()
    cfg = dict(sizes=tuple(int(x) for x in args.train_sizes.split(",")), max_raises=args.train_cap)
    res["train_abstraction"] = {"sizes_pct": list(cfg["sizes"]), "allin": True, "max_raises": cfg["max_raises"]}
    X, Y, M, _ = T.generate(seed=101, n=args.train, iters=args.iters, batch=args.gen_batch, log=log, **cfg)
    Xh, Yh, Mh, sh = T.generate(seed=202, n=args.heldout, iters=args.iters, batch=args.gen_batch, log=log, **cfg)
    res["generate_s"] = time.perf_counter() - t0
    net = P.LeafNet(P.LEAF_D_IN, args.width, args.depth, P.LEAF_D_OUT,
                    max_batch=max(args.batch, args.heldout, 1088))
    net.set_params(he_init(net, 0))
    t0 = time.perf_counter()
    hist = T.train(net, X, Y, M, steps=args.steps, batch=args.batch, lr=args.lr, log=log,
                   log_every=max(args.steps // 20, 1))
    torch.cuda.synchronize()
    res["train_s"] = time.perf_counter() - t0
    res["loss_history"] = hist
    pots = [s["pot"] for s, _ in sh]
    pred = net.forward(Xh).cpu().numpy()
    yh, mh, xh = Yh.cpu().numpy(), Mh.cpu().numpy(), Xh.cpu().numpy()
    e_net, _ = T.value_error_mbb(pred, yh, mh, xh, pots)
    m = M.cpu().numpy()
    const = (Y.cpu().numpy() * m).sum(axis=0) / np.maximum(m.sum(axis=0), 1)
    e_const, _ = T.value_error_mbb(np.broadcast_to(const, pred.shape), yh, mh, xh, pots)
    t_net = T.forward_ms(net, Xh)
    res["heldout_error_mbb_per_hand"] = {"network": e_net, "constant_predictor": e_const}
    res["network_ms_per_heldout_batch"] = t_net
    log(f"held-out error: network {e_net:.1f} mbb/hand, constant {e_const:.1f}; forward {t_net:.4f} ms")
    ks = [1, 2, 4, 8, 16, 32, 64, 128, 256]
    ks = [k for k in ks if k < args.iters]
    curve, ms_iter = T.plain_solver_curve(sh, Yh, Mh, Xh, ks)
    res["plain_solver"] = {"ms_per_batched_iteration": ms_iter, "error_mbb_per_hand_by_iterations": curve}
    k_eq = max(1, int(t_net // ms_iter))
    at_eq = min(curve, key=lambda kv: abs(kv[0] - k_eq))
    match = next((k for k, e in curve if e <= e_net), None)
    res["gain"] = {
        "plain_iterations_in_network_time": t_net / ms_iter,
        "plain_error_at_network_time_mbb": at_eq[1],
        "plain_iterations_to_match_network": match,
        "plain_ms_to_match_network": None if match is None else match * ms_iter,
        "time_ratio_at_equal_error": None if match is None else match * ms_iter / t_net,
    }
    log(f"plain solver: {curve}; {ms_iter:.4f} ms/iteration for the held-out batch")

    def save():
        if args.out:
            with open(args.out, "w") as f:
                f.write(json.dumps(res) + "\n")

    save()
    if args.flop:
        flop_comparison(net, 0, args.flop_iters, res)
        save()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
