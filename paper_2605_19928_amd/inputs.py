"""Seeded synthetic inputs: boards, private-hand ranges, pots and stacks.

This module holds no arithmetic of the solver.  It only draws random public
boards and range vectors with numpy's ``default_rng`` so that the GPU library
and the CPU oracle can be fed identical inputs.  Both sides import it; it
imports neither.

Conventions: card = 4*rank + suit (rank 0..12 = 2..A); a two-card combo
{a > b} has index a(a-1)/2 + b in [0, 1326).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

NCOMBO = 1326


def combo_cards() -> np.ndarray:
    """(1326, 2) array of (a, b) with a > b, row = combo index."""
    out = np.zeros((NCOMBO, 2), dtype=np.int32)
    for a in range(1, 52):
        for b in range(a):
            out[a * (a - 1) // 2 + b] = (a, b)
    return out


_CC = combo_cards()


def blocked_mask(board) -> np.ndarray:
    """Boolean (1326,) mask of combos that share a card with the board."""
    bset = np.zeros(52, dtype=bool)
    bset[np.asarray(board, dtype=np.int64)] = True
    return bset[_CC[:, 0]] | bset[_CC[:, 1]]


def draw_board(rng: np.random.Generator, n: int) -> list:
    return [int(c) for c in rng.choice(52, n, replace=False)]


def dirichlet_range(rng: np.random.Generator, board, alpha: float = 1.0, support: int | None = None) -> np.ndarray:
    """Symmetric Dirichlet(alpha) over the board-compatible combos.

    With ``support=k`` only k compatible combos, picked uniformly, get mass
    (the sparse-support ranges the per-history oracle can afford on big trees).
    """
    ok = np.flatnonzero(~blocked_mask(board))
    if support is not None:
        ok = np.sort(rng.choice(ok, size=min(support, ok.size), replace=False))
    w = rng.dirichlet(np.full(ok.size, alpha))
    r = np.zeros(NCOMBO, dtype=np.float64)
    r[ok] = w
    return r


def suit_stabilizer(board) -> list:
    """Suit permutations p (suit s -> p[s], tuples) mapping the board onto itself."""
    b = set(int(c) for c in board)
    return [p for p in itertools.permutations(range(4)) if {4 * (c // 4) + p[c % 4] for c in b} == b]


def symmetric_range(rng: np.random.Generator, board, alpha: float = 1.0, support: int | None = None) -> np.ndarray:
    """A range invariant under every suit permutation that fixes the board.

    The board-compatible combos fall into orbits under those permutations;
    Dirichlet(alpha) weights are drawn per orbit (``support=k``: only k
    orbits, picked uniformly, get mass) and every combo of an orbit carries
    its orbit's weight, then the range is scaled to sum 1, so combos of one
    orbit hold bitwise equal values."""
    cc = combo_cards()
    group = suit_stabilizer(board)
    blocked = blocked_mask(board)
    orbit = np.full(NCOMBO, -1)
    n_orb = 0
    for k in range(NCOMBO):
        if blocked[k] or orbit[k] >= 0:
            continue
        a, b = (int(x) for x in cc[k])
        for p in group:
            a2, b2 = 4 * (a // 4) + p[a % 4], 4 * (b // 4) + p[b % 4]
            hi, lo = max(a2, b2), min(a2, b2)
            orbit[hi * (hi - 1) // 2 + lo] = n_orb
        n_orb += 1
    live = np.arange(n_orb)
    if support is not None:
        live = np.sort(rng.choice(live, size=min(support, n_orb), replace=False))
    w = np.zeros(n_orb)
    w[live] = rng.dirichlet(np.full(live.size, alpha))
    r = np.zeros(NCOMBO, dtype=np.float64)
    ok = orbit >= 0
    r[ok] = w[orbit[ok]]
    return r / r.sum()


def draw_pot_stack(rng: np.random.Generator, spr_lo: float = 1.0, spr_hi: float = 8.0,
                   pot_lo: float = 20.0, pot_hi: float = 400.0, log_spr: bool = False):
    """Pot log-uniform in [pot_lo, pot_hi] rounded to an even chip count; stack = round(SPR * pot)."""
    pot = math.exp(rng.uniform(math.log(pot_lo), math.log(pot_hi)))
    pot = max(2, 2 * int(round(pot / 2)))
    if log_spr:
        spr = math.exp(rng.uniform(math.log(spr_lo), math.log(spr_hi)))
    else:
        spr = rng.uniform(spr_lo, spr_hi)
    stack = int(round(spr * pot))
    return pot, stack


def river_config(seed: int, support: int | None = None):
    """River subgame: 5-card board, Dirichlet(1) ranges, pot 100, stacks 400,
    sizes {50, 100}% + all-in, max 2 bets/raises per street."""
    rng = np.random.default_rng(seed)
    board = draw_board(rng, 5)
    r0 = dirichlet_range(rng, board, 1.0, support)
    r1 = dirichlet_range(rng, board, 1.0, support)
    spec = dict(board=board, pot=100, stacks=(400, 400), sizes=[50, 100], allin=True,
                max_raises=2, depth_limit=0)
    return spec, np.stack([r0, r1])


def turn_config(seed: int, support: int | None = None, spr: float | None = None, pot: int | None = None,
                sizes=(33, 75, 150), max_raises: int = 3):
    """Turn subgame solved to showdown: 4-card board, Dirichlet(1) ranges,
    pot log-uniform in [20, 400], SPR uniform in [1, 8] unless given,
    sizes {33, 75, 150}% + all-in, max 3 bets/raises per street."""
    rng = np.random.default_rng(seed)
    board = draw_board(rng, 4)
    r0 = dirichlet_range(rng, board, 1.0, support)
    r1 = dirichlet_range(rng, board, 1.0, support)
    p, st = draw_pot_stack(rng)
    if pot is not None:
        p = pot
    if spr is not None:
        st = int(round(spr * p))
    spec = dict(board=board, pot=p, stacks=(st, st), sizes=list(sizes), allin=True,
                max_raises=max_raises, depth_limit=0)
    return spec, np.stack([r0, r1])


def flop_config(seed: int, support: int | None = None, pot: int = 100, stack: int = 400,
                sizes=(33, 75), max_raises: int = 3):
    """Depth-limited flop subgame: 3-card board, Dirichlet(1) ranges, leaves at
    the turn card; pot 100, stack 400, sizes {33, 75}% + all-in, max 3."""
    rng = np.random.default_rng(seed)
    board = draw_board(rng, 3)
    r0 = dirichlet_range(rng, board, 1.0, support)
    r1 = dirichlet_range(rng, board, 1.0, support)
    spec = dict(board=board, pot=pot, stacks=(stack, stack), sizes=list(sizes), allin=True,
                max_raises=max_raises, depth_limit=1)
    return spec, np.stack([r0, r1])


def hand_classes() -> np.ndarray:
    """[1326] the preflop hand class of each combo: 0..12 pairs by rank, then
    suited and offsuit rank pairs (169 classes)."""
    cc = combo_cards()
    ra, rb = cc[:, 0] // 4, cc[:, 1] // 4
    hi, lo = np.maximum(ra, rb), np.minimum(ra, rb)
    pair_idx = hi * (hi - 1) // 2 + lo
    suited = cc[:, 0] % 4 == cc[:, 1] % 4
    return np.where(ra == rb, ra, 13 + np.where(suited, 0, 78) + pair_idx)


def preflop_config(seed: int, pot: int = 20, stack: int = 1000, sizes=(50, 100), max_raises: int = 3,
                   alpha: float = 1.0):
    """Preflop root (no board) stopping at the flop deal: pot 20 (each player
    in for 1 bb of 10 chips), 100 bb behind, sizes {50, 100}% without all-in,
    max 3 bets/raises.  Ranges are suit-symmetric: a Dirichlet(alpha) weight
    per hand class, spread evenly over the class's combos (uniform ranges are
    the true preflop start; these keep the symmetry and vary the mass)."""
    rng = np.random.default_rng(seed)
    cls = hand_classes()
    size = np.bincount(cls, minlength=169)
    r = []
    for _ in range(2):
        w = rng.dirichlet(np.full(169, alpha))
        r.append(w[cls] / size[cls])
    spec = dict(board=[], pot=pot, stacks=(stack, stack), sizes=list(sizes), allin=False,
                max_raises=max_raises, depth_limit=1)
    return spec, np.stack(r)


def batch_config(seed: int, count_nodes, n: int = 256, river_share: float = 0.7,
                 lo: int = 10, hi: int = 2000, sizes_pool=(33, 50, 75, 100, 150)):
    """Many independent river/turn subgames of uneven size.

    The first round(river_share * n) subgames are rivers, the rest turns.
    Each gets its own board, Dirichlet(1) ranges, pot (log-uniform [20, 400])
    and stack-to-pot ratio (uniform [1, 8]) and its own bet abstraction: 1-4
    sizes drawn from sizes_pool plus all-in, and 1-3 bets/raises per street.
    A draw is kept when count_nodes(spec), supplied by the caller, lies in
    [lo, hi]; otherwise the abstraction, pot and stack are drawn again.
    """
    rng = np.random.default_rng(seed)
    n_river = int(round(river_share * n))
    out = []
    for i in range(n):
        nb = 5 if i < n_river else 4
        board = draw_board(rng, nb)
        r0 = dirichlet_range(rng, board, 1.0)
        r1 = dirichlet_range(rng, board, 1.0)
        for _ in range(1000):
            k = int(rng.integers(1, 5))
            sizes = sorted(int(x) for x in rng.choice(sizes_pool, k, replace=False))
            cap = int(rng.integers(1, 4))
            pot, stack = draw_pot_stack(rng)
            spec = dict(board=board, pot=pot, stacks=(stack, stack), sizes=sizes, allin=True,
                        max_raises=cap, depth_limit=0)
            if lo <= count_nodes(spec) <= hi:
                break
        else:
            raise RuntimeError("no abstraction met the node-count window")
        out.append((spec, np.stack([r0, r1])))
    return out


def leaf_training_config(seed: int, index: int, sizes=(75,), max_raises: int = 2,
                         spr_lo: float = 0.1, spr_hi: float = 8.0):
    """One random turn subgame for leaf-network training data.

    Seeded by (seed, index): 4-card board; each player's range
    Dirichlet(alpha_p) over the compatible combos with alpha_p ~ U[0.5, 2];
    pot log-uniform in [20, 400] (even chips); stack-to-pot ratio
    log-uniform in [spr_lo, spr_hi] (the depth-limit leaves of a flop
    subgame sit at ratios from about 0.1 to 4); continuation abstraction
    {75}% + all-in, at most 2 bets/raises per street."""
    rng = np.random.default_rng([seed, index])
    board = draw_board(rng, 4)
    a0, a1 = rng.uniform(0.5, 2.0, size=2)
    r0 = dirichlet_range(rng, board, a0)
    r1 = dirichlet_range(rng, board, a1)
    pot, stack = draw_pot_stack(rng, spr_lo=spr_lo, spr_hi=spr_hi, log_spr=True)
    spec = dict(board=board, pot=pot, stacks=(stack, stack), sizes=list(sizes), allin=True,
                max_raises=max_raises, depth_limit=0)
    return spec, np.stack([r0, r1])
