"""Pins for the FP64 leaf-network reference (oracle/mlp.py).

* Backward pass vs central finite differences of the loss (no bf16 rounding).
* Huber loss gradient vs finite differences, both branches.
* Adam's first step has the closed form p - lr * g / (|g| + eps).
* bf16 rounding: round-to-nearest-even at the 16th mantissa bit, exact on
  representable values.
* Leaf inputs: each player's part sums to 1 and excludes combos holding the
  next card; one-hot board has 4 ones after a flop.
"""
import numpy as np

from oracle import mlp


def tiny(rng, d_in=7, width=5, depth=2, d_out=4):
    return [(rng.standard_normal((o, i)) * 0.5, rng.standard_normal(o) * 0.1)
            for o, i in mlp.layer_shapes(d_in, width, depth, d_out)]


def loss_of(params, x, t, m):
    y = mlp.forward(params, x, emulate_bf16=False)
    return mlp.huber_grad(y, t, m)[0]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    params = tiny(rng)
    x = rng.standard_normal((6, 7))
    t = rng.standard_normal((6, 4)) * 2
    m = (rng.random((6, 4)) > 0.2).astype(float)
    y, acts, pre = mlp.forward(params, x, emulate_bf16=False, return_acts=True)
    _, gy = mlp.huber_grad(y, t, m)
    grads = mlp.backward(params, acts, pre, gy, emulate_bf16=False)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for (i, j) in [(0, 0), (W.shape[0] - 1, W.shape[1] - 1), (1, 2)]:
            Wp = [(w.copy(), bb.copy()) for w, bb in params]
            Wm = [(w.copy(), bb.copy()) for w, bb in params]
            Wp[li][0][i, j] += h
            Wm[li][0][i, j] -= h
            fd = (loss_of(Wp, x, t, m) - loss_of(Wm, x, t, m)) / (2 * h)
            assert abs(fd - grads[li][0][i, j]) < 1e-6
        k = b.shape[0] - 1
        Bp = [(w.copy(), bb.copy()) for w, bb in params]
        Bm = [(w.copy(), bb.copy()) for w, bb in params]
        Bp[li][1][k] += h
        Bm[li][1][k] -= h
        fd = (loss_of(Bp, x, t, m) - loss_of(Bm, x, t, m)) / (2 * h)
        assert abs(fd - grads[li][1][k]) < 1e-6


def test_huber_gradient_both_branches():
    y = np.array([[0.3, 2.5, -4.0]])
    t = np.zeros((1, 3))
    m = np.ones((1, 3))
    loss, g = mlp.huber_grad(y, t, m)
    assert abs(loss - (0.5 * 0.09 + (2.5 - 0.5) + (4.0 - 0.5)) / 3) < 1e-15
    np.testing.assert_allclose(g, [[0.1, 1 / 3, -1 / 3]], atol=1e-15)


def test_adam_first_step_closed_form():
    p = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    g = [(np.array([[0.3, -1e-3]]), np.array([2.0]))]
    z = [(np.zeros((1, 2)), np.zeros(1))]
    lr = 1e-2
    out, m, v = mlp.adam_step(p, g, z, z, 1, lr)
    for (P0, G0), (P1,) in zip(((p[0][0], g[0][0]), (p[0][1], g[0][1])), ((out[0][0],), (out[0][1],))):
        np.testing.assert_allclose(P1, P0 - lr * G0 / (np.abs(G0) + 1e-8), rtol=1e-12)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.5, 0.0], dtype=np.float32)
    got = mlp.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1.0) wins; 1 + 3*2^-8 ties up to 1 + 2^-6
    np.testing.assert_array_equal(got, [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -3.5, 0.0])


def test_leaf_inputs_structure():
    rng = np.random.default_rng(3)
    board = [0, 17, 33]
    r = rng.random((2, 1326))
    cc = mlp.combo_cards()
    for b in board:
        r[:, (cc[:, 0] == b) | (cc[:, 1] == b)] = 0
    cards, X = mlp.leaf_inputs(r, board, pot=100, stack_behind=250, d_in=2705)
    assert len(cards) == 49 and X.shape == (49, 2705)
    for k, c in enumerate(cards):
        held = (cc[:, 0] == c) | (cc[:, 1] == c)
        for p in range(2):
            part = X[k, p * 1326:(p + 1) * 1326]
            assert abs(part.sum() - 1) < 1e-12 and not part[held].any()
        hot = X[k, 2652:2704]
        assert hot.sum() == 4 and hot[c] == 1 and all(hot[b] == 1 for b in board)
        assert X[k, 2704] == 2.5


def test_compatible_mass_brute_force():
    """M(h | c) against an explicit loop over opponent combos (sparse ranges)."""
    rng = np.random.default_rng(5)
    cc = mlp.combo_cards()
    r = np.zeros(1326)
    sup = rng.choice(1326, 40, replace=False)
    r[sup] = rng.random(40)
    card = 17
    m = mlp.compatible_mass(r, card)
    for h in rng.choice(1326, 60, replace=False):
        want = sum(r[o] for o in sup
                   if len({cc[h, 0], cc[h, 1], cc[o, 0], cc[o, 1]}) == 4 and card not in (cc[o, 0], cc[o, 1]))
        assert abs(m[h] - want) < 1e-12


def test_zero_sum_shift_closed_forms():
    """Constant outputs a, b shift by (a + b) / 2 (the two joint masses are
    equal); after any shift the weighted values of both players cancel."""
    rng = np.random.default_rng(6)
    cc = mlp.combo_cards()
    board = [3, 20, 41]
    ok = ~np.isin(cc, board).any(axis=1)
    reach = np.zeros((2, 1326))
    reach[:, ok] = rng.random((2, ok.sum()))
    card = 9
    ev = np.stack([np.full(1326, 0.3), np.full(1326, -0.1)])
    assert abs(mlp.zero_sum_shift(ev, reach, card) - 0.1) < 1e-12
    ev = rng.standard_normal((2, 1326))
    d = mlp.zero_sum_shift(ev, reach, card)
    keep = (cc[:, 0] != card) & (cc[:, 1] != card)
    m1 = mlp.compatible_mass(reach[1], card)
    m0 = mlp.compatible_mass(reach[0], card)
    total = ((reach[0] * keep) * m1 * (ev[0] - d)).sum() + ((reach[1] * keep) * m0 * (ev[1] - d)).sum()
    assert abs(total) < 1e-9 * ((reach[0] * m1).sum())


def test_zero_sum_shifts_batched_equals_per_row():
    rng = np.random.default_rng(4)
    board = [3, 17, 40]
    from paper_2605_19928_amd import inputs as I
    reach = np.stack([I.dirichlet_range(rng, board), I.dirichlet_range(rng, board, support=30)])
    cards = [c for c in range(52) if c not in board][:7]
    ev = rng.standard_normal((len(cards), 2, 1326))
    got = mlp.zero_sum_shifts(ev, reach, cards)
    want = [mlp.zero_sum_shift(ev[j], reach, c) for j, c in enumerate(cards)]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)
