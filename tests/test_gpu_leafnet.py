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
  At full size (2705 -> 4 x 1536 -> 2652, batch 1024): three steps, each
  step's loss, the first step's gradients, and the parameters after three
  steps against Adam's recursion fed with the GPU's gradients.
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


def close(g, o, name, fro_max=1e-3, rel_max=5e-3):
    g = np.asarray(g, np.float64).ravel()
    o = np.asarray(o, np.float64).ravel()
    rel = np.abs(g - o).max() / max(np.abs(o).max(), 1e-30)
    fro = np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-300)
    cos = float(g @ o / (np.linalg.norm(g) * np.linalg.norm(o) + 1e-300))
    say(f"  {name}: max rel err {rel:.2e}, frobenius rel err {fro:.2e}, cosine {cos:.8f}")
    assert fro <= fro_max and cos > 0.9999 and rel <= rel_max


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


def test_train_steps_full_size_gradients_and_adam_moments():
    """The leaf architecture at its training batch (2705 -> 4 x 1536 -> 2652,
    1024 rows): three train steps on one batch.  Each step's loss against
    the FP64 forward with bf16 emulation under the GPU's current parameters
    (so the bf16 weight copies written after each update are checked too),
    the first step's gradients against the FP64 backward (the forward's
    bounds, except 1e-2 relative for the input layer's weight gradient), and
    the parameters after three steps against the oracle's Adam recursion in
    FP64 (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments) fed with
    the GPU's own gradients of each step.

    The input layer's weight gradient is the product of the deepest
    back-propagated gradient, rounded to bf16 after each of four layers: the
    same reference with the same bf16 roundings but float32 sums (what the
    GPU accumulates in) moves it by 3.6e-3 relative (Frobenius and largest
    entry) on this case, and the other layers' by at most 4e-4 and 1e-3."""
    import torch
    m = 1024
    say(f"case: train steps at full size d_in={P.LEAF_D_IN} width=1536 depth=4 d_out={P.LEAF_D_OUT} m={m}")
    rng = np.random.default_rng(8)
    net = P.LeafNet(P.LEAF_D_IN, 1536, 4, P.LEAF_D_OUT, max_batch=m)
    params = rand_params(rng, net.layer_shapes(), scale=1.4)
    net.set_params(params)
    x = (rng.standard_normal((m, P.LEAF_D_IN)) * 0.5).astype(np.float32)
    t = rng.standard_normal((m, P.LEAF_D_OUT)).astype(np.float32)
    mk = (rng.random((m, P.LEAF_D_OUT)) > 0.2).astype(np.float32)
    xt, tt, mt = (torch.from_numpy(a).cuda() for a in (x, t, mk))
    lr = 1e-3
    p_ref = [(W.astype(np.float64), b.astype(np.float64)) for W, b in params]
    m_ref = [(np.zeros_like(W), np.zeros_like(b)) for W, b in p_ref]
    v_ref = [(np.zeros_like(W), np.zeros_like(b)) for W, b in p_ref]
    cur = params
    for step in range(1, 4):
        loss = net.train_step(xt, tt, mt, lr)
        y, acts, pre = mlp.forward(cur, x, emulate_bf16=True, return_acts=True)
        ref_loss, gy = mlp.huber_grad(y, t, mk)
        say(f"  step {step}: loss gpu {loss:.8f} ref {ref_loss:.8f}")
        assert abs(loss - ref_loss) <= 1e-4 * max(abs(ref_loss), 1)
        g = net.get_grads()
        if step == 1:
            grads = mlp.backward(cur, acts, pre, gy, emulate_bf16=True)
            for li, ((gW, gb), (rW, rb)) in enumerate(zip(g, grads)):
                close(gW, rW, f"dW layer {li}", **({"fro_max": 1e-2, "rel_max": 1e-2} if li == 0 else {}))
                close(gb, rb, f"db layer {li}")
        g64 = [(gW.astype(np.float64), gb.astype(np.float64)) for gW, gb in g]
        p_ref, m_ref, v_ref = mlp.adam_step(p_ref, g64, m_ref, v_ref, step, lr)
        cur = net.get_params()
    worst = 0.0
    for (W, b), (rW, rb) in zip(cur, p_ref):
        for a, r in ((W, rW), (b, rb)):
            np.testing.assert_allclose(a, r, rtol=1e-5, atol=1e-7)
            worst = max(worst, float(np.abs(a - r).max()))
    say(f"  parameters after 3 Adam steps: max |d| = {worst:.3e}")


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
