"""Pins for oracle parts that the GPU parity tests lean on and that nothing
else fixes: the table-driven depth-limit leaf value, the current-strategy
reach of every node, the network forward pass and Adam's moment
accumulation.

* Leaf values (Sec. 3, the depth-limited game: a leaf's value to a hand is
  the pot times the value the leaf model assigns per unit of pot, averaged
  over the next public card, per history).  On a flop tree where both
  players can only check, the root value has closed forms:
  constant EV e_i gives pot * e_i * M_{-i}(h), with M the opponent mass
  compatible with h; EV equal to the card's index gives the mean of the
  indices of the 45 cards that neither hand nor the board holds, written
  here as (1326 - sum of used cards) / 45; a per-hand EV g_i(h) gives
  pot * g_i(h) * M_{-i}(h).  On a full betting tree an antisymmetric table
  (EV_1 = -EV_0 = const) keeps the root values zero-sum every iteration.
* Reach under the current strategy: for every node, the root range times
  the product of the actor's regret-matching probabilities along the path,
  with hands holding a card dealt on the path at zero.
* Network forward: a hand-computed 2-layer ReLU network, with and without
  bf16 operand rounding.
* Adam: under a constant gradient the bias-corrected moments are g and g^2
  at every step, so each step moves a parameter by lr * g / (|g| + eps).
"""
import numpy as np
import pytest

import oracle as O
from oracle import mlp
from paper_2605_19928_amd import inputs as I

CC = I.combo_cards()


def compat_matrix():
    a, b = CC[:, 0], CC[:, 1]
    share = (a[:, None] == a[None, :]) | (a[:, None] == b[None, :]) | (b[:, None] == a[None, :]) | \
            (b[:, None] == b[None, :])
    return (~share).astype(np.float64)


def checkcheck_flop(seed):
    rng = np.random.default_rng(seed)
    board = I.draw_board(rng, 3)
    r = np.stack([I.dirichlet_range(rng, board, 1.0, 60), I.dirichlet_range(rng, board, 1.0, 60)])
    spec = dict(board=board, pot=60, stacks=(200, 200), sizes=[], allin=False, max_raises=0, depth_limit=1)
    return spec, r


def solve_one_iteration(spec, r, table):
    t = O.Tree.holdem(**spec)
    s = O.Solver(t, r)
    assert s.num_leaves() == 1
    s.set_leaf_table(table)
    s.iterate(1)
    return t, s


def test_checkcheck_tree_is_one_leaf():
    spec, _ = checkcheck_flop(0)
    t = O.Tree.holdem(**spec)
    e = t.export()
    assert list(e["type"]) == [O.T_DEC, O.T_DEC, O.T_LEAF]
    assert list(e["contrib"][2]) == [30, 30]


@pytest.mark.parametrize("seed", [0, 1])
def test_leaf_table_constant_ev(seed):
    spec, r = checkcheck_flop(seed)
    e = np.array([0.37, -1.25])
    table = np.zeros((1, 2, 52, 1326))
    table[0, 0] = e[0]
    table[0, 1] = e[1]
    _, s = solve_one_iteration(spec, r, table)
    v = s.root_cfv("current")
    K = compat_matrix()
    ok = ~I.blocked_mask(spec["board"])
    for i in range(2):
        want = spec["pot"] * e[i] * (K @ r[1 - i])
        np.testing.assert_allclose(v[i][ok], want[ok], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 2])
def test_leaf_table_card_index_ev(seed):
    """EV(h | c) = c for both players: the leaf averages over the 45 cards
    neither the board nor either hand holds."""
    spec, r = checkcheck_flop(seed)
    table = np.zeros((1, 2, 52, 1326))
    table[0, :, :, :] = np.arange(52, dtype=np.float64)[None, :, None]
    _, s = solve_one_iteration(spec, r, table)
    v = s.root_cfv("current")
    K = compat_matrix()
    ok = ~I.blocked_mask(spec["board"])
    bsum = float(sum(spec["board"]))
    hsum = (CC[:, 0] + CC[:, 1]).astype(np.float64)
    for i in range(2):
        ro = r[1 - i]
        # sum over compatible ho of r_o(ho) * (1326 - board - cards(h) - cards(ho)) / 45
        want = ((1326.0 - bsum - hsum) * (K @ ro) - K @ (ro * hsum)) / 45.0 * spec["pot"]
        np.testing.assert_allclose(v[i][ok], want[ok], rtol=1e-12, atol=1e-12)


def test_leaf_table_per_hand_ev_uses_the_traversers_hand():
    spec, r = checkcheck_flop(3)
    rng = np.random.default_rng(9)
    g = rng.standard_normal((2, 1326))
    table = np.zeros((1, 2, 52, 1326))
    table[0] = g[:, None, :]
    _, s = solve_one_iteration(spec, r, table)
    v = s.root_cfv("current")
    K = compat_matrix()
    ok = ~I.blocked_mask(spec["board"])
    for i in range(2):
        want = spec["pot"] * g[i] * (K @ r[1 - i])
        np.testing.assert_allclose(v[i][ok], want[ok], rtol=1e-12, atol=1e-12)


def test_leaf_table_antisymmetric_zero_sum_on_betting_tree():
    """Every leaf pays pot * e to player 0 and -pot * e to player 1 per
    compatible pair, folds and showdowns are zero-sum: the reach-weighted
    root values cancel at every iteration, whatever the strategies."""
    spec, r = I.flop_config(4, support=50)
    t = O.Tree.holdem(**spec)
    s = O.Solver(t, r)
    nl = s.num_leaves()
    assert nl > 1
    table = np.zeros((nl, 2, 52, 1326))
    table[:, 0] = 0.4
    table[:, 1] = -0.4
    s.set_leaf_table(table)
    for _ in range(4):
        s.iterate(1)
        v = s.root_cfv("current")
        total = (r[0] * v[0]).sum() + (r[1] * v[1]).sum()
        scale = np.abs(r[0] * v[0]).sum() + np.abs(r[1] * v[1]).sum()
        assert scale > 0 and abs(total) <= 1e-12 * scale


def path_reach(tree, solver, ranges):
    """Reach of both players at every node by walking each node's path to the root."""
    e = tree.export()
    n = tree.n_nodes
    cur = {}
    out = np.zeros((n, 2, 1326))
    for node in range(n):
        rr = ranges.copy()
        c = node
        while e["parent"][c] >= 0:
            p = int(e["parent"][c])
            if e["type"][p] == O.T_DEC:
                if p not in cur:
                    cur[p] = solver.strategy(p, "current")
                rr[int(e["player"][p])] *= cur[p][int(e["action"][c])]
            elif e["type"][p] == O.T_CHANCE:
                card = int(e["chance_card"][c])
                rr[:, (CC[:, 0] == card) | (CC[:, 1] == card)] = 0.0
            c = p
        out[node] = rr
    return out


@pytest.mark.parametrize("which", ["river", "turn"])
def test_reach_current_is_the_path_product(which):
    if which == "river":
        spec, r = I.river_config(2, support=80)
    else:
        spec, r = I.turn_config(3, support=30, spr=1.0, sizes=(75,), max_raises=2)
    t = O.Tree.holdem(**spec)
    if which == "turn":
        assert t.n_chance > 0
    s = O.Solver(t, r)
    s.iterate(3)
    got = s.reach_current()
    want = path_reach(t, s, r)
    ok = ~I.blocked_mask(spec["board"])
    np.testing.assert_allclose(got[:, :, ok], want[:, :, ok], rtol=1e-13, atol=1e-300)


def test_mlp_forward_hand_computed():
    W1 = np.array([[1.0, -1.0], [2.0, 0.5], [0.25, 0.25]])
    b1 = np.array([0.0, -1.0, -2.0])
    W2 = np.array([[1.0, 3.0, 5.0], [-0.5, 0.0, 1.0]])
    b2 = np.array([0.5, -0.25])
    params = [(W1, b1), (W2, b2)]
    x = np.array([[1.0, 2.0], [-2.0, 4.0]])
    # row 0: z1 = (-1, 2+1-1, 0.75-2) -> relu (0, 2, 0) -> y = (0.5 + 6, -0.25 + 0)
    # row 1: z1 = (-6, -4+2-1, -0.5+1-2) -> relu (0, 0, 0) -> y = (0.5, -0.25)
    want = np.array([[6.5, -0.25], [0.5, -0.25]])
    np.testing.assert_array_equal(mlp.forward(params, x, emulate_bf16=False), want)
    np.testing.assert_array_equal(mlp.forward(params, x, emulate_bf16=True), want)
    # bf16 rounding applies to the input: 1 + 2^-9 rounds to 1 (ties to even)
    x2 = np.array([[1.0 + 2.0 ** -9, 2.0]])
    np.testing.assert_array_equal(mlp.forward(params, x2, emulate_bf16=True), want[:1])
    y = mlp.forward(params, x2, emulate_bf16=False)
    # without rounding z1[1] = 2(1 + 2^-9) + 1 - 1 = 2 + 2^-8, y0 = 0.5 + 3 * (2 + 2^-8)
    assert y[0, 0] == 0.5 + 3 * (2 + 2.0 ** -8)


def test_adam_constant_gradient_steps():
    p = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    g = [(np.array([[0.3, -4.0]]), np.array([1e-3]))]
    m = [(np.zeros((1, 2)), np.zeros(1))]
    v = [(np.zeros((1, 2)), np.zeros(1))]
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        p, m, v = mlp.adam_step(p, g, m, v, t, lr, eps=eps)
        for (pw, pb), (gw, gb), (mw, mb), (vw, vb), p0 in zip(p, g, m, v, [(np.array([[1.0, -2.0]]), np.array([0.5]))]):
            np.testing.assert_allclose(mw, (1 - 0.9 ** t) * gw, rtol=1e-12)
            np.testing.assert_allclose(vw, (1 - 0.999 ** t) * gw * gw, rtol=1e-12)
            np.testing.assert_allclose(pw, p0[0] - t * lr * gw / (np.abs(gw) + eps), rtol=1e-12)
            np.testing.assert_allclose(pb, p0[1] - t * lr * gb / (np.abs(gb) + eps), rtol=1e-12)
