"""Pins for the oracle's online pruning (Sec. 5): the dominance test and the
reduced game.

* With no flag set the reduced tree is the tree itself.
* Reduction bookkeeping: every kept node keeps its attributes, parents map to
  parents, and the node count drops by the sizes of the removed subtrees.
* Soundness on Kuhn poker: when the second player holds only the king,
  folding to a bet is dominated (calling wins every showdown); the reduced
  game has the full game's value, -1 chip per hand for the first player in
  closed form (checking and giving up is the best the first player can do).
* Soundness on a hold'em river where the second player holds only the nuts
  (a royal flush with the ten of spades): folding is dominated at every node
  where that player faces a bet.  Both games are solved; the value of a
  two-player zero-sum game lies in [-BR_1, BR_0] for any strategy profile, so
  the two brackets must overlap, and both hold the closed-form value (the
  first player loses its half of the pot).
* Properties of the test on random bounds: no decision node loses every
  action, narrowing the intervals never brings an action back, and a player
  with an empty range prunes nothing.
"""
import numpy as np
import pytest

import oracle as O

ALPHA, BETA, GAMMA = 1.5, 0.0, 2.0


def _river():
    # A-K-Q-J of spades and the deuce of hearts: the ten of spades is a royal flush
    board = [51, 47, 43, 39, 2]
    return O.Tree.holdem(board, 20, (100, 100), [50, 100], allin=True, max_raises=2), board


def _subtree_sizes(e):
    n = len(e["type"])
    size = np.ones(n, dtype=np.int64)
    for v in range(n - 1, 0, -1):
        size[e["parent"][v]] += size[v]
    return size


def _bracket(tree, ranges, iters):
    s = O.Solver(tree, ranges, ALPHA, BETA, GAMMA)
    s.iterate(iters)
    _, br = s.exploitability()
    return -br[1], br[0]


def test_no_flags_is_identity():
    t, _ = _river()
    r, m = t.prune(np.zeros(t.n_nodes, dtype=np.uint8))
    assert r.n_nodes == t.n_nodes and np.array_equal(m, np.arange(t.n_nodes))
    a, b = t.export(), r.export()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_reduction_bookkeeping():
    t, _ = _river()
    e = t.export()
    rng = np.random.default_rng(3)
    flags = np.zeros(t.n_nodes, dtype=np.uint8)
    for n in np.flatnonzero(e["type"] == O.T_DEC):
        fc, A = int(e["first_child"][n]), int(e["n_child"][n])
        if A >= 2 and rng.random() < 0.5:
            flags[fc + rng.integers(A)] = 1
    r, new = t.prune(flags)
    f = r.export()
    size = _subtree_sizes(e)
    # flags inside an already removed subtree remove nothing more
    inside = np.zeros(t.n_nodes, dtype=bool)
    for v in range(1, t.n_nodes):
        inside[v] = inside[e["parent"][v]] or flags[e["parent"][v]] == 1
    top = (flags == 1) & ~inside
    assert (flags & inside).any() and r.n_nodes == t.n_nodes - int(size[top].sum())
    kept = np.flatnonzero(new >= 0)
    assert len(kept) == r.n_nodes and np.array_equal(new[kept], np.arange(r.n_nodes))
    for k in ("type", "player", "depth", "chance_card"):
        assert np.array_equal(f[k], e[k][kept]), k
    assert np.array_equal(f["contrib"], e["contrib"][kept])
    par = e["parent"][kept]
    assert f["parent"][0] == -1 and np.array_equal(f["parent"][1:], new[par[1:]])
    for n in np.flatnonzero(e["type"] == O.T_DEC):
        ch = [int(c) for c in range(e["first_child"][n], e["first_child"][n] + e["n_child"][n]) if new[c] >= 0]
        m = new[n]
        assert f["n_child"][m] == len(ch)
        assert list(range(f["first_child"][m], f["first_child"][m] + f["n_child"][m])) == [int(new[c]) for c in ch]
    # boards survive the reduction
    for n in kept[:: max(1, len(kept) // 50)]:
        assert r.node_board(int(new[n])) == t.node_board(int(n))


def test_invalid_flags_rejected():
    t, _ = _river()
    e = t.export()
    flags = np.zeros(t.n_nodes, dtype=np.uint8)
    flags[0] = 1                                   # the root has no parent action
    with pytest.raises(ValueError):
        t.prune(flags)
    flags[:] = 0
    n = int(np.flatnonzero(e["type"] == O.T_DEC)[0])
    flags[e["first_child"][n]: e["first_child"][n] + e["n_child"][n]] = 1   # every action of a node
    with pytest.raises(ValueError):
        t.prune(flags)


def test_kuhn_king_never_folds():
    k = O.Tree.kuhn_poker()
    e = k.export()
    ranges = np.array([[1.0, 1.0, 1.0], [0.0, 0.0, 1.0]])
    lo = np.full((k.n_nodes, 3), -np.inf)
    hi = np.full((k.n_nodes, 3), np.inf)
    # node 2: the second player facing a bet; children 5 (fold, -1) and 6 (call, +2 with the king)
    lo[5, 2], hi[5, 2] = -1.0, -1.0
    lo[6, 2], hi[6, 2] = 2.0, 2.0
    flags = k.prune_dominated(ranges, lo, hi)
    assert list(np.flatnonzero(flags)) == [5]
    r, new = k.prune(flags)
    assert r.n_nodes == 8 and r.export()["n_child"][new[2]] == 1
    lo_f, hi_f = _bracket(k, ranges, 4000)
    lo_r, hi_r = _bracket(r, ranges, 4000)
    for lo_v, hi_v in ((lo_f, hi_f), (lo_r, hi_r)):
        assert lo_v - 1e-3 <= -1.0 <= hi_v + 1e-3
    # with the queen also in the range the fold is no longer dominated for every hand
    ranges2 = np.array([[1.0, 1.0, 1.0], [0.0, 1.0, 1.0]])
    lo[5, 1], hi[5, 1] = -1.0, -1.0
    lo[6, 1], hi[6, 1] = -2.0, 2.0
    assert not k.prune_dominated(ranges2, lo, hi).any()


def test_river_nuts_never_fold():
    t, board = _river()
    e = t.export()
    nh = O.NCOMBO
    ten = 4 * 8 + 3
    ranges = np.zeros((2, nh))
    ranges[0, np.random.default_rng(5).choice(nh, 200, replace=False)] = 1.0
    for c in range(52):
        if c != ten and c not in board:
            a, b = max(c, ten), min(c, ten)
            ranges[1, a * (a - 1) // 2 + b] = 1.0
    lo = np.full((t.n_nodes, nh), -np.inf)
    hi = np.full((t.n_nodes, nh), np.inf)
    facing = 0
    for n in np.flatnonzero((e["type"] == O.T_DEC) & (e["player"] == 1)):
        fc = int(e["first_child"][n])
        c = e["contrib"][n]
        if c[0] > c[1]:                        # facing a bet: fold, call, raises
            facing += 1
            lo[fc], hi[fc] = -c[1], -c[1]      # folding loses what is in
            lo[fc + 1], hi[fc + 1] = c[0], c[0]   # calling wins the bet with the nuts
    flags = t.prune_dominated(ranges, lo, hi)
    removed = np.flatnonzero(flags)
    assert facing > 0 and len(removed) == facing
    assert all(e["type"][x] == O.T_FOLD and e["player"][e["parent"][x]] == 1 for x in removed)
    r, _ = t.prune(flags)
    assert r.n_nodes == t.n_nodes - facing
    lo_f, hi_f = _bracket(t, ranges, 200)
    lo_r, hi_r = _bracket(r, ranges, 200)
    print(f"brackets: full [{lo_f:.4f}, {hi_f:.4f}] reduced [{lo_r:.4f}, {hi_r:.4f}]")
    assert hi_f - lo_f < 0.5 and hi_r - lo_r < 0.5
    assert max(lo_f, lo_r) <= min(hi_f, hi_r) + 1e-9
    # closed form: against the nuts the first player gives up its half of the pot
    assert lo_f - 1e-3 <= -10.0 <= hi_f + 1e-3 and lo_r - 1e-3 <= -10.0 <= hi_r + 1e-3


def test_dominance_properties():
    t, board = _river()
    e = t.export()
    nh = O.NCOMBO
    rng = np.random.default_rng(7)
    ranges = rng.random((2, nh)) * (rng.random((2, nh)) < 0.05)
    mid = rng.normal(size=(t.n_nodes, nh)) * 10
    # narrow intervals so that dominance occurs on some public actions
    for n in np.flatnonzero(e["type"] == O.T_DEC):
        fc, A = int(e["first_child"][n]), int(e["n_child"][n])
        mid[fc: fc + A] += rng.normal(size=(A, 1)) * 40
    half = rng.random((t.n_nodes, nh)) * 5
    lo, hi = mid - half, mid + half
    flags = t.prune_dominated(ranges, lo, hi)
    assert flags.any()
    for n in np.flatnonzero(e["type"] == O.T_DEC):
        fc, A = int(e["first_child"][n]), int(e["n_child"][n])
        assert flags[fc: fc + A].sum() < A
    t.prune(flags)          # accepted
    # narrower intervals remove a superset
    lo2, hi2 = lo + half * 0.5, hi - half * 0.5
    flags2 = t.prune_dominated(ranges, lo2, hi2)
    assert np.all(flags2 >= flags)
    # an actor with no hand removes nothing at its nodes
    r0 = ranges.copy()
    r0[1] = 0
    f0 = t.prune_dominated(r0, lo, hi)
    assert not any(f0[c] for n in np.flatnonzero((e["type"] == O.T_DEC) & (e["player"] == 1))
                   for c in range(e["first_child"][n], e["first_child"][n] + e["n_child"][n]))
