"""Pins for the oracle's CFR machinery on Kuhn poker.

* Game value -1/18 for the first player (Kuhn 1950) and exploitability going
  to zero under DCFR.
* The second player's equilibrium strategy is unique: after a check it bets
  the jack with probability 1/3 (and always the king), facing a bet it calls
  the queen with probability 1/3 (always the king, never the jack).
* The first two DCFR iterations match a brute-force enumeration of Kuhn's
  histories written independently below (regrets, both discount branches, and
  the average-strategy weights).
"""
import numpy as np
import pytest

import oracle as O

ALPHA, BETA, GAMMA = 1.5, 0.0, 2.0


@pytest.fixture(scope="module")
def kuhn():
    return O.Tree.kuhn_poker()


def test_tree_shape(kuhn):
    e = kuhn.export()
    assert kuhn.n_nodes == 9 and kuhn.n_decision == 4 and kuhn.n_fold == 2 and kuhn.n_showdown == 3
    assert list(e["type"]) == [0, 0, 0, 2, 0, 1, 2, 1, 2]
    assert list(e["player"][[0, 1, 2, 4]]) == [0, 1, 1, 0]


def test_value_and_exploitability(kuhn):
    s = O.Solver(kuhn, np.ones((2, 3)), ALPHA, BETA, GAMMA)
    s.iterate(10000)
    expl, br = s.exploitability()
    assert 0 <= expl < 1e-3
    v = s.root_cfv("avg")
    game_value = (v[0] * 1.0).sum() / s.pair_mass()
    assert abs(game_value + 1 / 18) < 1e-3
    # zero-sum: player 1's value is the negation
    assert abs((v[1]).sum() / s.pair_mass() - 1 / 18) < 1e-3
    # BR values bracket the game value
    assert br[0] >= game_value - 1e-12 and br[1] >= -game_value - 1e-12


def test_second_player_equilibrium(kuhn):
    s = O.Solver(kuhn, np.ones((2, 3)), ALPHA, BETA, GAMMA)
    s.iterate(10000)
    after_check = s.strategy(1, "avg")     # actions: check, bet; hands J, Q, K
    facing_bet = s.strategy(2, "avg")      # actions: fold, call
    assert abs(after_check[1, 0] - 1 / 3) < 0.02
    assert after_check[1, 1] < 0.02 and after_check[1, 2] > 0.98
    assert abs(facing_bet[1, 1] - 1 / 3) < 0.02
    assert facing_bet[1, 0] < 0.02 and facing_bet[1, 2] > 0.98


# ---------------------------------------------------------------- brute force
# Histories over {c, b, f}: '' P0, 'c' P1, 'b' P1, 'cb' P0.  Terminal:
# 'cc' showdown for 1, 'bc'/'cbc' showdown for 2, 'bf' P1 folds, 'cbf' P0 folds.
INFOSETS = {"": ("c", "b"), "c": ("c", "b"), "b": ("f", "c"), "cb": ("f", "c")}
NODE_OF = {"": 0, "c": 1, "b": 2, "cb": 4}      # breadth-first ids of the oracle tree
ACTOR = {"": 0, "c": 1, "b": 1, "cb": 0}


def payoff0(h, c0, c1):
    win = 1 if c0 > c1 else -1
    if h == "cc":
        return win
    if h in ("bc", "cbc"):
        return 2 * win
    if h == "bf":
        return 1
    if h == "cbf":
        return -1
    raise KeyError(h)


def value(h, c0, c1, sig, i):
    """Expected utility for player i from history h (both cards known)."""
    if h not in INFOSETS:
        u = payoff0(h, c0, c1)
        return u if i == 0 else -u
    p = ACTOR[h]
    card = c0 if p == 0 else c1
    return sum(sig[(h, card)][k] * value(h + a, c0, c1, sig, i) for k, a in enumerate(INFOSETS[h]))


def reach(h, c, sig, p):
    """Player p's own reach of history h holding card c."""
    pr = 1.0
    for j in range(len(h)):
        pre = h[:j]
        if ACTOR[pre] == p:
            pr *= sig[(pre, c)][INFOSETS[pre].index(h[j])]
    return pr


def brute_iteration(sig):
    """Instantaneous regrets and reach-weighted strategy for every infoset."""
    reg, sadd = {}, {}
    for h, acts in INFOSETS.items():
        p = ACTOR[h]
        for c in range(3):
            r = np.zeros(len(acts))
            for o in range(3):
                if o == c:
                    continue
                c0, c1 = (c, o) if p == 0 else (o, c)
                w = reach(h, o, sig, 1 - p)
                v = value(h, c0, c1, sig, p)
                for k, a in enumerate(acts):
                    r[k] += w * (value(h + a, c0, c1, sig, p) - v)
            reg[(h, c)] = r
            sadd[(h, c)] = reach(h, c, sig, p) * np.array(sig[(h, c)])
    return reg, sadd


def rm(R):
    pos = np.maximum(R, 0)
    return pos / pos.sum() if pos.sum() > 0 else np.full(len(R), 1 / len(R))


def test_first_two_dcfr_iterations_match_brute_force(kuhn):
    s = O.Solver(kuhn, np.ones((2, 3)), ALPHA, BETA, GAMMA)
    R = {k: np.zeros(2) for k in ((h, c) for h in INFOSETS for c in range(3))}
    S = {k: np.zeros(2) for k in R}
    for t in (1, 2):
        sig = {k: rm(R[k]) for k in R}
        reg, sadd = brute_iteration(sig)
        dpos = t ** ALPHA / (t ** ALPHA + 1)
        dneg = t ** BETA / (t ** BETA + 1)
        for k in R:
            x = R[k] + reg[k]
            R[k] = np.where(x > 0, x * dpos, x * dneg)
            S[k] = (S[k] + sadd[k]) * (t / (t + 1)) ** GAMMA
        s.iterate(1)
        Ro, So = s.rows("R"), s.rows("S")
        rows_of = {0: 0, 1: 2, 2: 4, 4: 6}
        for (h, c), v in R.items():
            row = rows_of[NODE_OF[h]]
            np.testing.assert_allclose(Ro[row:row + 2, c], v, atol=1e-14)
            np.testing.assert_allclose(So[row:row + 2, c], S[(h, c)], atol=1e-14)
    # iteration 2 exercised both discount branches
    assert any((v > 0).any() for v in R.values()) and any((v < 0).any() for v in R.values())


@pytest.mark.parametrize("variant,bound", [("cfr+", 2e-3), ("pcfr+", 1e-5)])
def test_variants_reach_the_game_value(kuhn, variant, bound):
    s = O.Solver(kuhn, np.ones((2, 3)), variant=variant)
    s.iterate(5000)
    e, _ = s.exploitability()
    v = s.root_cfv("avg")
    assert 0 <= e < bound
    assert abs(v[0].sum() / s.pair_mass() + 1 / 18) < max(bound, 1e-6)


@pytest.mark.parametrize("variant", ["cfr+", "pcfr+"])
def test_variant_first_iterations_match_brute_force(kuhn, variant):
    """CFR+ floors regrets at 0 and weights the average by t; PCFR+ also
    matches on R + m with m the previous instantaneous regret and weights the
    average by t^2 (Tammelin 2014; Farina, Kroer & Sandholm 2021)."""
    s = O.Solver(kuhn, np.ones((2, 3)), variant=variant)
    R = {k: np.zeros(2) for k in ((h, c) for h in INFOSETS for c in range(3))}
    S = {k: np.zeros(2) for k in R}
    M = {k: np.zeros(2) for k in R}
    rows_of = {0: 0, 1: 2, 2: 4, 4: 6}
    for t in (1, 2, 3):
        sig = {k: rm(R[k] + (M[k] if variant == "pcfr+" else 0)) for k in R}
        reg, sadd = brute_iteration(sig)
        for k in R:
            R[k] = np.maximum(R[k] + reg[k], 0.0)
            S[k] = S[k] + (t if variant == "cfr+" else t * t) * sadd[k]
            M[k] = reg[k]
        s.iterate(1)
        Ro, So = s.rows("R"), s.rows("S")
        for (h, c), v in R.items():
            row = rows_of[NODE_OF[h]]
            np.testing.assert_allclose(Ro[row:row + 2, c], v, atol=1e-14)
            np.testing.assert_allclose(So[row:row + 2, c], S[(h, c)], atol=1e-14)
        for node in (0, 1, 2, 4):
            cur = s.strategy(node, "current")
            for c in range(3):
                key = next(h for h in INFOSETS if NODE_OF[h] == node)
                want = rm(R[(key, c)] + (M[(key, c)] if variant == "pcfr+" else 0))
                np.testing.assert_allclose(cur[:, c], want, atol=1e-14)


@pytest.mark.parametrize("variant", ["dcfr", "cfr+", "pcfr+"])
def test_alternating_first_iterations_match_brute_force(kuhn, variant):
    """Alternating updates: within iteration t player 0 is updated from
    sigma^t, then player 1 against player 0's new strategy (regret matching
    of the updated regrets, plus the prediction for PCFR+); both halves use
    iteration t's discounts and touch only their own player's rows."""
    s = O.Solver(kuhn, np.ones((2, 3)), variant=variant, alternating=True)
    R = {k: np.zeros(2) for k in ((h, c) for h in INFOSETS for c in range(3))}
    S = {k: np.zeros(2) for k in R}
    M = {k: np.zeros(2) for k in R}
    rows_of = {0: 0, 1: 2, 2: 4, 4: 6}
    for t in (1, 2, 3):
        for upd in (0, 1):
            sig = {k: rm(R[k] + (M[k] if variant == "pcfr+" else 0)) for k in R}
            reg, sadd = brute_iteration(sig)
            for k in R:
                if ACTOR[k[0]] != upd:
                    continue
                x = R[k] + reg[k]
                if variant == "dcfr":
                    R[k] = np.where(x > 0, x * t ** ALPHA / (t ** ALPHA + 1), x * t ** BETA / (t ** BETA + 1))
                    S[k] = (S[k] + sadd[k]) * (t / (t + 1)) ** GAMMA
                else:
                    R[k] = np.maximum(x, 0.0)
                    S[k] = S[k] + (t if variant == "cfr+" else t * t) * sadd[k]
                    M[k] = reg[k]
        s.iterate(1)
        Ro, So = s.rows("R"), s.rows("S")
        for (h, c), v in R.items():
            row = rows_of[NODE_OF[h]]
            np.testing.assert_allclose(Ro[row:row + 2, c], v, atol=1e-14)
            np.testing.assert_allclose(So[row:row + 2, c], S[(h, c)], atol=1e-14)


def test_alternating_reaches_the_game_value(kuhn):
    s = O.Solver(kuhn, np.ones((2, 3)), ALPHA, BETA, GAMMA, alternating=True)
    s.iterate(5000)
    e, _ = s.exploitability()
    assert 0 <= e < 1e-3
    assert abs(s.root_cfv("avg")[0].sum() / s.pair_mass() + 1 / 18) < 1e-3


# ---------------------------------------------------------------- dynamic thresholding
THR0 = 0.08


def rm_thr(R, thr):
    """Regret matching, then probabilities below thr set to 0 and the rest renormalised."""
    q = rm(R)
    q = np.where(q < thr, 0.0, q)
    return q / q.sum()


def test_thresholded_iterations_match_brute_force(kuhn):
    """Dynamic thresholding (cited in Sec. 2): iteration t matches on the
    regrets, drops every action below thr0 / sqrt(t) and renormalises.  The
    first 25 DCFR iterations against the brute-force enumeration, with the
    threshold applied there independently; some action falls below it."""
    s = O.Solver(kuhn, np.ones((2, 3)), ALPHA, BETA, GAMMA, threshold=THR0)
    R = {k: np.zeros(2) for k in ((h, c) for h in INFOSETS for c in range(3))}
    S = {k: np.zeros(2) for k in R}
    cut = 0
    for t in range(1, 26):
        thr = THR0 / np.sqrt(t)
        sig = {k: rm_thr(R[k], thr) for k in R}
        cut += sum(int(((rm(R[k]) > 0) & (sig[k] == 0)).any()) for k in R)
        reg, sadd = brute_iteration(sig)
        dpos = t ** ALPHA / (t ** ALPHA + 1)
        dneg = t ** BETA / (t ** BETA + 1)
        for k in R:
            x = R[k] + reg[k]
            R[k] = np.where(x > 0, x * dpos, x * dneg)
            S[k] = (S[k] + sadd[k]) * (t / (t + 1)) ** GAMMA
        s.iterate(1)
        Ro, So = s.rows("R"), s.rows("S")
        rows_of = {0: 0, 1: 2, 2: 4, 4: 6}
        for (h, c), v in R.items():
            row = rows_of[NODE_OF[h]]
            np.testing.assert_allclose(Ro[row:row + 2, c], v, atol=1e-13)
            np.testing.assert_allclose(So[row:row + 2, c], S[(h, c)], atol=1e-13)
        # the current strategy the oracle reports is the one iteration t + 1 will use
        for (h, c) in R:
            np.testing.assert_allclose(s.strategy(NODE_OF[h], "current")[:, c],
                                       rm_thr(R[(h, c)], THR0 / np.sqrt(t + 1)), atol=1e-14)
    assert cut > 0


def test_thresholded_dcfr_reaches_the_game_value(kuhn):
    s = O.Solver(kuhn, np.ones((2, 3)), ALPHA, BETA, GAMMA, threshold=THR0)
    s.iterate(10000)
    expl, _ = s.exploitability()
    v = s.root_cfv("avg")
    assert 0 <= expl < 1e-3
    assert abs(v[0].sum() / s.pair_mass() + 1 / 18) < 1e-3
