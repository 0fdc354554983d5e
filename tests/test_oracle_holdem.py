"""Pins for the oracle on hold'em subgames.

* Tree shape of the river configuration (pot 100, stacks 400, {50,100}% +
  all-in, at most two bets/raises per street).
* Showdown values of a check-down river tree equal brute-force pairwise sums
  of sign(value difference) over compatible opponent hands (Sec. 4.3 Stage 4
  defines the showdown value; the brute force is the O(n^2) sum it replaces).
* A check-down turn tree equals brute force over the 44 river cards each pair
  leaves (the chance weighting of Stage 6).
* Zero-sum: sum_h r0 v0 + sum_h r1 v1 = 0 at the root for every sigma^t.
* Best-response values bracket the game value; exploitability >= 0 and falls.
* Relabelling suits permutes every output the same way.
* The all-in/stub-leaf equity table is antisymmetric and matches a
  brute-force runout average.
"""
import numpy as np
import pytest

import oracle as O
from paper_2605_19928_amd import inputs as I

CC = I.combo_cards()


def ranks_on(board):
    """Seven-card value of every combo on a five-card board (-1 if blocked)."""
    bm = I.blocked_mask(board)
    hands = np.zeros((1326, 7), dtype=np.int32)
    hands[:, :2] = CC
    hands[:, 2:] = board
    v = O.eval7_batch(hands)
    v[bm] = -1
    return v


def compat_matrix():
    a = np.zeros((1326, 52), dtype=bool)
    a[np.arange(1326), CC[:, 0]] = True
    a[np.arange(1326), CC[:, 1]] = True
    return ~(a.astype(np.int32) @ a.T.astype(np.int32)).astype(bool)


COMPAT = compat_matrix()


def test_river_tree_shape():
    spec, _ = I.river_config(0)
    t = O.Tree.holdem(**spec)
    e = t.export()
    assert (t.n_nodes, t.n_decision, t.n_fold, t.n_showdown, t.n_chance) == (51, 18, 16, 17, 0)
    assert list(np.bincount(e["depth"])) == [1, 4, 15, 21, 10]
    assert t.n_rows == 50
    kids = range(e["first_child"][0], e["first_child"][0] + e["n_child"][0])
    # check, bet 50, bet 100, all-in 400 (contributions include the 50 each already in)
    assert [tuple(e["contrib"][k]) for k in kids] == [(50, 50), (100, 50), (150, 50), (450, 50)]
    # facing a pot-size bet of 100 (contrib 150 vs 50): fold, call, raise 50%, raise 100%, all-in
    n = e["first_child"][0] + 2
    kids = range(e["first_child"][n], e["first_child"][n] + e["n_child"][n])
    got = [tuple(e["contrib"][k]) for k in kids]
    assert got[0] == (150, 50) and got[1] == (150, 150)
    # the pot after calling is 300: a 50% raise puts in 100 + 150 -> 300 total; a 100% raise
    # puts in 100 + 300 -> 450, the cap, which merges with the all-in; the bet count (2) is used up
    assert got[2:] == [(150, 300), (150, 450)]
    assert e["n_child"][n] == 4


def test_checkdown_river_is_pairwise_equity():
    rng = np.random.default_rng(3)
    board = I.draw_board(rng, 5)
    r = np.stack([I.dirichlet_range(rng, board), I.dirichlet_range(rng, board)])
    t = O.Tree.holdem(board, 100, (400, 400), [50], allin=False, max_raises=0)
    assert (t.n_nodes, t.n_decision, t.n_showdown) == (3, 2, 1)
    s = O.Solver(t, r)
    s.iterate(1)
    v = s.root_cfv("current")
    rk = ranks_on(board)
    ok = rk >= 0
    sign = np.sign(rk[:, None] - rk[None, :]) * (COMPAT & ok[:, None] & ok[None, :])
    np.testing.assert_allclose(v[0], 50 * sign @ r[1], atol=1e-12)
    np.testing.assert_allclose(v[1], 50 * sign @ r[0], atol=1e-12)


def test_checkdown_turn_averages_44_rivers():
    rng = np.random.default_rng(4)
    board = I.draw_board(rng, 4)
    r = np.stack([I.dirichlet_range(rng, board, support=40), I.dirichlet_range(rng, board, support=40)])
    t = O.Tree.holdem(board, 60, (0, 0), [50], allin=False, max_raises=0)
    assert t.n_chance == 1 and t.n_showdown == 48
    s = O.Solver(t, r)
    s.iterate(1)
    v = s.root_cfv("current")
    want = np.zeros((2, 1326))
    for card in range(52):
        if card in board:
            continue
        rk = ranks_on(board + [card])
        ok = rk >= 0
        sign = np.sign(rk[:, None] - rk[None, :]) * (COMPAT & ok[:, None] & ok[None, :])
        want[0] += 30 * sign @ r[1] / 44
        want[1] += 30 * sign @ r[0] / 44
    np.testing.assert_allclose(v, want, atol=1e-12)


@pytest.fixture(scope="module")
def small_river():
    spec, r = I.river_config(11, support=70)
    t = O.Tree.holdem(**spec)
    return t, r


def test_zero_sum_every_iteration(small_river):
    t, r = small_river
    s = O.Solver(t, r)
    for _ in range(6):
        s.iterate(1)
        v = s.root_cfv("current")
        total = (r[0] * v[0]).sum() + (r[1] * v[1]).sum()
        scale = np.abs(r[0] * v[0]).sum()
        assert abs(total) <= 1e-12 * max(scale, 1.0)


def test_best_response_brackets_and_decreases(small_river):
    t, r = small_river
    s = O.Solver(t, r)
    prev = None
    for n in (5, 20, 80):
        s.iterate(n - s.t)
        e, br = s.exploitability()
        v = s.root_cfv("avg")
        gv = (r[0] * v[0]).sum() / s.pair_mass()
        assert br[0] >= gv - 1e-9 and br[1] >= -gv - 1e-9
        assert e >= 0
        if prev is not None:
            assert e < prev
        prev = e


def test_suit_relabelling_permutes_outputs():
    spec, r = I.river_config(5, support=60)
    perm_suit = np.array([2, 0, 3, 1])
    cmap = np.array([4 * (c // 4) + perm_suit[c % 4] for c in range(52)])
    # combo index after relabelling
    a, b = cmap[CC[:, 0]], cmap[CC[:, 1]]
    hi, lo = np.maximum(a, b), np.minimum(a, b)
    cidx = hi * (hi - 1) // 2 + lo
    r2 = np.zeros_like(r)
    r2[:, cidx] = r
    spec2 = dict(spec, board=[int(cmap[c]) for c in spec["board"]])
    t1, t2 = O.Tree.holdem(**spec), O.Tree.holdem(**spec2)
    s1, s2 = O.Solver(t1, r), O.Solver(t2, r2)
    s1.iterate(15)
    s2.iterate(15)
    v1, v2 = s1.root_cfv("current"), s2.root_cfv("current")
    np.testing.assert_allclose(v2[:, cidx], v1, atol=1e-10)
    for node in (0, 3, 7):
        np.testing.assert_allclose(s2.strategy(node)[:, cidx], s1.strategy(node), atol=1e-10)


def test_equity_table_turn_board():
    rng = np.random.default_rng(9)
    board = I.draw_board(rng, 4)
    t = O.Tree.holdem(board, 100, (400, 400), [75], allin=True, max_raises=1, depth_limit=1)
    e = t.export()
    leaf = int(np.flatnonzero(e["type"] == O.T_LEAF)[0])
    E = t.equity_table(leaf)
    np.testing.assert_allclose(E, -E.T, atol=1e-15)
    # brute force over the 44 rivers for a few pairs
    ok = np.flatnonzero(~I.blocked_mask(board))
    pick = rng.choice(ok, 6, replace=False)
    per_river = {c: ranks_on(board + [c]) for c in range(52) if c not in board}
    for h in pick:
        for o in pick:
            if not COMPAT[h, o]:
                continue
            vals = [np.sign(rk[h] - rk[o]) for c, rk in per_river.items()
                    if c not in CC[h] and c not in CC[o]]
            assert len(vals) == 44
            assert abs(E[h, o] - np.mean(vals)) < 1e-15
