"""Preflop roots (no board) in the oracle: the depth-limited tree whose
leaves sit at the flop deal, the canonical flops that stand for their suit
orbits (the lossless suit abstraction, Sec. 4.5, applied to the flop), and
the value of a preflop leaf -- pinned to published counts, to brute force
and to the symmetry that makes 169 hand classes lossless.

A preflop leaf's value for a history (h, o) is pot x the mean, over the
C(48, 3) = 17296 flops clear of both hands, of the expected value E(h | g);
a flop g takes its value from the table row of its canonical flop f, the
hand mapped back, averaged over the permutations that carry f to g."""
import itertools

import numpy as np
import pytest

import oracle as O
from oracle import mlp

CC = mlp.combo_cards()
PERMS = list(itertools.permutations(range(4)))


def pcard(p, c):
    return 4 * (c // 4) + p[c % 4]


def fmask(cards):
    return sum(1 << int(c) for c in cards)


def canon(m):
    cards = [c for c in range(52) if m >> c & 1]
    return min(fmask(pcard(p, c) for c in cards) for p in PERMS)


def preflop_tree(**kw):
    spec = dict(board=[], pot=20, stacks=(1000, 1000), sizes=[100], allin=False, max_raises=1, depth_limit=1)
    spec.update(kw)
    return O.Tree.holdem(**spec)


def test_canonical_flops_are_the_1755_suit_classes():
    cards, orbit = O.canonical_flops()
    # the 22100 flops fall into 1755 strategically distinct classes
    assert len(cards) == 1755 and int(orbit.sum()) == 22100
    flops = list(itertools.combinations(range(52), 3))
    cmap = {}
    for f in flops:
        c = canon(fmask(f))
        cmap[c] = cmap.get(c, 0) + 1
    want = sorted(cmap, key=lambda m: [c for c in range(52) if m >> c & 1])   # by sorted cards
    got = [fmask(c) for c in cards]
    assert got == want
    assert [cmap[m] for m in want] == orbit.tolist()
    # trips flops: 13 classes of 4 flops each
    trips = [k for k, c in enumerate(cards) if c[0] // 4 == c[1] // 4 == c[2] // 4]
    assert len(trips) == 13 and set(orbit[trips]) == {4}


def test_preflop_tree_shape_and_refusals():
    t = preflop_tree()
    e = t.export()
    # root check/bet; after a check the second player checks (leaf) or bets
    # (then fold / call); after a bet, fold or call: 9 nodes, 3 leaves
    assert e["type"].tolist() == [O.T_DEC, O.T_DEC, O.T_DEC, O.T_LEAF, O.T_DEC, O.T_FOLD, O.T_LEAF, O.T_FOLD,
                                  O.T_LEAF]
    assert e["contrib"].tolist() == [[10, 10], [10, 10], [30, 10], [10, 10], [10, 30], [30, 10], [30, 30],
                                     [10, 30], [30, 30]]
    assert t.flop_leaves and t.n_leaf == 3
    with pytest.raises(ValueError):        # an all-in would need a five-card runout
        preflop_tree(allin=True)
    with pytest.raises(ValueError):        # a preflop root must stop at the flop
        preflop_tree(depth_limit=0)
    with pytest.raises(ValueError):        # raises capped at a small stack put a player all in
        preflop_tree(stacks=(15, 15))


def brute_leaf_value(tab, pot, hi, ho, cards):
    """pot x mean over flops clear of both hands of E(hi | g)."""
    canon_index = {fmask(c): k for k, c in enumerate(cards)}
    used = set(CC[hi]) | set(CC[ho])
    tot, n = 0.0, 0
    for g in itertools.combinations([c for c in range(52) if c not in used], 3):
        gm = fmask(g)
        cm = canon(gm)
        f = canon_index[cm]
        fc = [c for c in range(52) if cm >> c & 1]
        vals = []
        for p in PERMS:
            if fmask(pcard(p, c) for c in fc) != gm:
                continue
            inv = [p.index(s) for s in range(4)]
            a, b = (pcard(inv, int(c)) for c in CC[hi])
            vals.append(tab[f][max(a, b) * (max(a, b) - 1) // 2 + min(a, b)])
        tot += np.mean(vals)
        n += 1
    assert n == 17296
    return pot * tot / n


def test_preflop_leaf_value_matches_brute_force_over_flops():
    t = preflop_tree()
    s = O.Solver(t, np.ones((2, 1326)))
    rng = np.random.default_rng(4)
    ev = rng.standard_normal((s.num_leaves(), 2, 1755, 1326))
    s.set_flop_leaf_table(ev)
    cards, _ = O.canonical_flops()
    e = t.export()
    leaves = np.flatnonzero(e["type"] == O.T_LEAF)
    for li, hi, ho, i in [(0, 5, 900, 0), (2, 1325, 17, 1), (1, 333, 1000, 0)]:
        n = int(leaves[li])
        pot = float(e["contrib"][n].sum())
        onehot = np.zeros(1326)
        onehot[ho] = 1.0
        got = s.leaf_cfv(n, i, onehot)[hi]
        want = brute_leaf_value(ev[li, i], pot, hi, ho, cards)
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (li, hi, ho, got, want)


def class_of():
    a, b = CC[:, 0], CC[:, 1]
    ra, rb = a // 4, b // 4
    hi, lo = np.maximum(ra, rb), np.minimum(ra, rb)
    kind = np.where(ra == rb, 0, np.where(a % 4 == b % 4, 1, 2))
    key = (hi * 13 + lo) * 3 + kind
    _, cls = np.unique(key, return_inverse=True)
    return cls


@pytest.mark.parametrize("symmetric", ["uniform", "by class"])
def test_preflop_leaf_cfv_is_the_class_sum_over_canonical_flops(symmetric):
    """With suit-symmetric opponent reach, a hand's leaf value is the class
    formula: pot / 17296 / |c| x sum over canonical flops f of orbit(f) x the
    sum over the class's combos x clear of f of E(x | f) M(x | f)."""
    cls = class_of()
    assert cls.max() + 1 == 169
    rng = np.random.default_rng(8)
    ro = np.ones(1326) if symmetric == "uniform" else rng.random(169)[cls]
    t = preflop_tree()
    s = O.Solver(t, np.ones((2, 1326)))
    ev = rng.standard_normal((s.num_leaves(), 2, 1755, 1326))
    s.set_flop_leaf_table(ev)
    cards, orbit = O.canonical_flops()
    e = t.export()
    n = int(np.flatnonzero(e["type"] == O.T_LEAF)[1])
    pot = float(e["contrib"][n].sum())
    got = s.leaf_cfv(n, 1, ro)
    K = ((CC[:, 0][:, None] != CC[:, 0][None, :]) & (CC[:, 0][:, None] != CC[:, 1][None, :]) &
         (CC[:, 1][:, None] != CC[:, 0][None, :]) & (CC[:, 1][:, None] != CC[:, 1][None, :])).astype(float)
    acc = np.zeros(169)
    for f in range(1755):
        keep = np.ones(1326, dtype=bool)
        for c in cards[f]:
            keep &= (CC[:, 0] != c) & (CC[:, 1] != c)
        M = K @ (ro * keep)
        acc += orbit[f] * np.bincount(cls, weights=ev[1, 1, f] * M * keep, minlength=169)
    size = np.bincount(cls, minlength=169)
    want = pot / 17296 * (acc / size)[cls]
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())


def test_preflop_iterates_stay_suit_symmetric():
    """From suit-symmetric ranges the preflop game is symmetric, so every
    iterate is constant over each of the 169 hand classes."""
    cls = class_of()
    rng = np.random.default_rng(2)
    r = np.stack([rng.random(169)[cls], rng.random(169)[cls]])
    t = preflop_tree(sizes=[50, 100], max_raises=2)
    s = O.Solver(t, r)
    s.set_flop_leaf_table(rng.standard_normal((s.num_leaves(), 2, 1755, 1326)))
    s.iterate(3)
    e = t.export()
    for n in np.flatnonzero(e["type"] == O.T_DEC):
        for which in ("current", "avg"):
            st = s.strategy(int(n), which)
            for c in range(169):
                blk = st[:, cls == c]
                assert np.abs(blk - blk[:, :1]).max() <= 1e-12, (n, which, c)
    v = s.root_cfv("current")
    for c in range(169):
        assert np.ptp(v[:, cls == c], axis=1).max() <= 1e-9 * np.abs(v).max()


def test_flop_zero_sum_shift_makes_each_row_zero_sum():
    """After the shift, sum_h r0 M1 (EV0 - d) + r1 M0 (EV1 - d) = 0 for each
    flop row, with M summed over opponent combos one by one."""
    rng = np.random.default_rng(6)
    reach = rng.random((2, 1326))
    flops = np.array([[0, 1, 2], [3, 17, 40]])
    ev = rng.standard_normal((2, 2, 1326))
    d = mlp.flop_zero_sum_shifts(ev, reach, flops)
    cards = [set(int(c) for c in CC[h]) for h in range(1326)]
    for j, f in enumerate(flops):
        fs = set(int(c) for c in f)
        clear = [h for h in range(1326) if not cards[h] & fs]
        m = {p: np.zeros(1326) for p in (0, 1)}
        for h in clear:
            opp = [o for o in clear if not cards[o] & cards[h]]
            m[1][h] = reach[1, opp].sum()
            m[0][h] = reach[0, opp].sum()
        z = sum(reach[0, h] * m[1][h] * (ev[j, 0, h] - d[j]) + reach[1, h] * m[0][h] * (ev[j, 1, h] - d[j])
                for h in clear)
        scale = sum(reach[0, h] * m[1][h] for h in clear)
        assert abs(z) <= 1e-9 * scale
