"""Leaf network and depth-limited solving on the GPU vs the FP64 references.

* Forward GEMM chain (bf16 MFMA, FP32 accumulate) vs oracle/mlp.py with the
  same bf16 roundings: relative error in Frobenius norm <= 1e-3, cosine
  similarity > 0.9999, and every entry within 5e-3 of the output scale, on
  ragged shapes and on the full leaf architecture (2705 -> 4 x 1536 -> 2652)
  at 1029 rows.  (A hidden activation whose FP32 and FP64 sums straddle a
  bf16 rounding boundary rounds one bf16 ulp apart, ~0.4%, so single
  entries of a deep network move more than the norm does.)
* One training step: gradients vs the FP64 backward with bf16 emulation
  (same bounds); the Adam update vs the closed form of Adam's first step.
* Depth-limited flop with exact check-down leaves, FP64: 1e-9 pot vs the
  oracle; FP32 within 1e-4 pot on values.
* Depth-limited flop with a network at the leaves: the oracle builds the leaf
  inputs from its own reach, runs the FP64 network, and values the leaves
  history by history; 1e-4 pot after 3 iterations.
"""
import numpy as np
import pytest

import oracle as O
from oracle import mlp
from paper_2605_19928_amd import inputs as I
from paper_2605_19928_amd import pcfr as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rand_params(rng, shapes, scale=1.0):
    return [((rng.standard_normal((o, i)) * scale / np.sqrt(i)).astype(np.float32),
             (rng.standard_normal(o) * 0.05).astype(np.float32)) for o, i in shapes]


def close(g, o, name):
    g = np.asarray(g, np.float64).ravel()
    o = np.asarray(o, np.float64).ravel()
    rel = np.abs(g - o).max() / max(np.abs(o).max(), 1e-30)
    fro = np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-300)
    cos = float(g @ o / (np.linalg.norm(g) * np.linalg.norm(o) + 1e-300))
    say(f"  {name}: max rel err {rel:.2e}, frobenius rel err {fro:.2e}, cosine {cos:.8f}")
    assert fro <= 1e-3 and cos > 0.9999 and rel <= 5e-3


@pytest.mark.parametrize("d_in,width,depth,d_out,m", [(300, 256, 2, 200, 130), (2705, 1536, 4, 2652, 1029)])
def test_forward_matches_fp64_reference(d_in, width, depth, d_out, m):
    import torch
    say(f"case: forward d_in={d_in} width={width} depth={depth} d_out={d_out} m={m}")
    rng = np.random.default_rng(d_in + m)
    net = P.LeafNet(d_in, width, depth, d_out, max_batch=m)
    params = rand_params(rng, net.layer_shapes(), scale=1.5)
    net.set_params(params)
    x = rng.standard_normal((m, d_in)).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = mlp.forward(params, x, emulate_bf16=True)
    close(y, ref, "forward")


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_forward_each_gemm_tile_matches_fp64_reference(tile):
    """Every forward GEMM tile, on a row count (1029 -> 1088) that leaves the
    last 128-row tile half empty, against the bf16-emulating FP64 reference."""
    import torch
    # direct tiles read their input in the layout the layer before writes, so
    # never on the first layer; they also serve the output layer
    say(f"case: forward with GEMM tile {tile} on every layer it fits, m=1029")
    rng = np.random.default_rng(77)
    net = P.LeafNet(P.LEAF_D_IN, 1536, 2, P.LEAF_D_OUT, max_batch=1029)
    params = rand_params(rng, net.layer_shapes(), scale=1.5)
    net.set_params(params)
    L = len(net.layer_shapes())
    tiles = [0] + [tile] * (L - 1) if tile >= 8 else [tile] * L
    net.tiles = tiles
    assert net.tiles == tiles
    if tile >= 8:
        with pytest.raises(P.PcfrError):
            net.tiles = [tile] * L                   # not on the first layer
        with pytest.raises(P.PcfrError):
            net.tiles = [0, tile] + [0] * (L - 2)    # a direct layer feeds direct layers only
        assert net.tiles == tiles
    x = rng.standard_normal((1029, P.LEAF_D_IN)).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    close(y, mlp.forward(params, x, emulate_bf16=True), f"forward tile {tile}")


def test_forward_after_autotune():
    import torch
    rng = np.random.default_rng(78)
    net = P.LeafNet(P.LEAF_D_IN, 1536, 4, P.LEAF_D_OUT, max_batch=1029)
    params = rand_params(rng, net.layer_shapes(), scale=1.5)
    net.set_params(params)
    before, after = net.autotune(1029, 3)
    say(f"case: GEMM tile autotune m=1029: {before:.4f} -> {after:.4f} ms per forward, tiles {net.tiles}")
    assert before > 0 and after > 0 and all(t in range(11) for t in net.tiles)
    x = rng.standard_normal((1029, P.LEAF_D_IN)).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    close(y, mlp.forward(params, x, emulate_bf16=True), "forward after autotune")
    with pytest.raises(P.PcfrError):
        net.tiles = [3] * (len(net.layer_shapes()) - 1)


def test_train_step_gradients_and_adam():
    import torch
    d_in, width, depth, d_out, m = 200, 192, 2, 130, 100
    say(f"case: train step d_in={d_in} width={width} depth={depth} d_out={d_out} m={m}")
    rng = np.random.default_rng(5)
    net = P.LeafNet(d_in, width, depth, d_out, max_batch=m)
    params = rand_params(rng, net.layer_shapes(), scale=1.5)
    net.set_params(params)
    x = rng.standard_normal((m, d_in)).astype(np.float32)
    t = (rng.standard_normal((m, d_out)) * 2).astype(np.float32)
    mk = (rng.random((m, d_out)) > 0.3).astype(np.float32)
    lr = 1e-3
    loss = net.train_step(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), torch.from_numpy(mk).cuda(), lr)
    y, acts, pre = mlp.forward(params, x, emulate_bf16=True, return_acts=True)
    ref_loss, gy = mlp.huber_grad(y, t, mk)
    say(f"  loss gpu {loss:.8f} ref {ref_loss:.8f}")
    assert abs(loss - ref_loss) <= 1e-4 * max(abs(ref_loss), 1)
    grads = mlp.backward(params, acts, pre, gy, emulate_bf16=True)
    g = net.get_grads()
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(g, grads)):
        close(gW, rW, f"dW layer {li}")
        close(gb, rb, f"db layer {li}")
    # Adam's first step: p - lr * g / (|g| + eps), with the GPU's own gradients
    newp = net.get_params()
    for (W0, b0), (W1, b1), (gW, gb) in zip(params, newp, g):
        for p0, p1, gg in ((W0, W1, gW), (b0, b1, gb)):
            want = p0.astype(np.float64) - lr * gg / (np.abs(gg) + 1e-8)
            np.testing.assert_allclose(p1, want, rtol=1e-5, atol=1e-7)


def flop_case(support=150, seed=0):
    spec, r = I.flop_config(seed, support=support)
    return spec, r


@pytest.mark.parametrize("dtype,T", [("f64", 30), ("f32", 30)])
def test_flop_depth_limited_exact_leaves(dtype, T):
    spec, r = flop_case()
    say(f"case: flop depth-limited, exact leaves, {spec} T={T} {dtype}")
    ot = O.Tree.holdem(**spec)
    os_ = O.Solver(ot, r)
    os_.iterate(T)
    gt = P.Tree(**spec)
    assert (gt.n_leaf, gt.n_allin) == (21, 14)
    gs = P.Solver(gt, r, P.SolverConfig(dtype=dtype))
    gs.iterate(T)
    pot = spec["pot"]
    tol = 1e-9 if dtype == "f64" else 1e-4
    ok = ~I.blocked_mask(spec["board"])
    d = np.abs(gs.root_cfv("current") - os_.root_cfv("current"))[:, ok].max() / pot
    say(f"  root cfv (current) max |d| = {d:.3e} pot")
    assert d <= tol
    da = np.abs(gs.root_cfv("avg") - os_.root_cfv("avg"))[:, ok].max() / pot
    eg, _ = gs.exploitability()
    eo, _ = os_.exploitability()
    say(f"  root cfv (avg) max |d| = {da:.3e} pot; exploitability gpu {eg:.9f} oracle {eo:.9f}")
    assert da <= tol and abs(eg - eo) / pot <= tol
    if dtype == "f64":
        e = gt.export()
        for n in np.flatnonzero(e["type"] == P.NODE_DECISION):
            assert np.abs(gs.strategy(int(n)) - os_.strategy(int(n)))[:, ok].max() <= 1e-9


def turn_leaf_case(support=120, seed=3):
    """Depth-limited turn (leaves at the river card): 4-card board, so the
    network rows carry four board cards plus the next card and there are 48
    next cards per leaf."""
    rng = np.random.default_rng(seed)
    board = I.draw_board(rng, 4)
    r = np.stack([I.dirichlet_range(rng, board, 1.0, support), I.dirichlet_range(rng, board, 1.0, support)])
    spec = dict(board=board, pot=100, stacks=(400, 400), sizes=[50, 100], allin=True, max_raises=2, depth_limit=1)
    return spec, r


@pytest.mark.parametrize("street,zero_sum", [("flop", True), ("flop", False), ("turn", True)])
def test_flop_depth_limited_network_leaves(street, zero_sum):
    import torch
    spec, r = flop_case(support=120, seed=1) if street == "flop" else turn_leaf_case()
    say(f"case: {street} depth-limited, network leaves, zero-sum correction {zero_sum}, {spec}")
    rng = np.random.default_rng(9)
    gt = P.Tree(**spec)
    gs = P.Solver(gt, r, P.SolverConfig(dtype="f64"))
    n_leaves, n_next = gs.leaf_rows()
    if street == "flop":
        assert (n_leaves, n_next) == (21, 49)
    else:
        assert n_leaves > 0 and n_next == 48
    net = P.LeafNet(P.LEAF_D_IN, 64, 2, P.LEAF_D_OUT, max_batch=n_leaves * n_next)
    params = rand_params(rng, net.layer_shapes(), scale=2.0)
    net.set_params(params)
    gs.attach_leafnet(net)
    gs.set_leaf_zero_sum(zero_sum)
    ot = O.Tree.holdem(**spec)
    os_ = O.Solver(ot, r)
    e = ot.export()
    leaves = np.flatnonzero(e["type"] == O.T_LEAF)
    eff = spec["stacks"][0]
    T = 3
    for it in range(T):
        reach = os_.reach_current()
        ev = np.zeros((len(leaves), 2, 52, 1326))
        for li, n in enumerate(leaves):
            c = e["contrib"][n][0]
            cards, X = mlp.leaf_inputs(reach[n], spec["board"], pot=2 * c, stack_behind=spec["pot"] // 2 + eff - c,
                                       d_in=P.LEAF_D_IN)
            Y = mlp.forward(params, X, emulate_bf16=True)
            for k, card in enumerate(cards):
                row = np.stack([Y[k, :1326], Y[k, 1326:]])
                if zero_sum:
                    row = row - mlp.zero_sum_shift(row, reach[n], card)
                ev[li, 0, card] = row[0]
                ev[li, 1, card] = row[1]
        os_.set_leaf_table(ev)
        os_.iterate(1)
        gs.iterate(1)
        d = np.abs(gs.root_cfv("current") - os_.root_cfv("current"))[:, ~I.blocked_mask(spec["board"])].max()
        say(f"  iteration {it + 1}: root cfv (current) max |d| = {d / spec['pot']:.3e} pot")
        assert d / spec["pot"] <= 1e-4
