"""FP64 reference for the leaf value network and its depth-limit leaf inputs.

TEST INFRASTRUCTURE (same rules as the rest of ``oracle/``).

The paper values depth-limit leaves with a network f_theta of the players'
normalised reach probabilities and the public state (Sec. 3, the
depth-limited solving equation; Sec. 4.2 Stage 2 builds the batched input
matrix X, Sec. 4.3 Stage 5 evaluates it in one batch).  It gives no
architecture; the one used here is a plain MLP with ReLU hidden layers.

Everything is computed in float64.  ``bf16`` rounds a float32 value to the
nearest bfloat16 (ties to even), which is what the GPU does to the operands
it multiplies; applying it here to the same operands makes the FP64 result
differ from the GPU's only by float32 accumulation.
"""
from __future__ import annotations

import numpy as np

NCOMBO = 1326


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layer_shapes(d_in: int, width: int, depth: int, d_out: int):
    dims = [d_in] + [width] * depth + [d_out]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def forward(params, x, emulate_bf16: bool = True, return_acts: bool = False):
    """y = W_L relu(... relu(W_1 x + b_1) ...) + b_L, row-major batches.

    params: list of (W [out, in], b [out]) float arrays (float32 masters).
    With emulate_bf16 the input, the weights and every hidden activation are
    rounded to bfloat16 before they are multiplied; sums are exact-ish FP64.
    """
    q = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    h = q(x)
    acts = [h]
    pre = []
    for i, (W, b) in enumerate(params):
        z = h @ q(W).T + np.asarray(b, dtype=np.float64)
        pre.append(z)
        if i + 1 < len(params):
            h = q(np.maximum(z, 0.0))
            acts.append(h)
        else:
            h = z
    return (h, acts, pre) if return_acts else h


def huber_grad(y, t, mask, delta=1.0):
    """Mean Huber loss over masked entries and its gradient w.r.t. y."""
    d = (y - t) * mask
    a = np.abs(d)
    loss_el = np.where(a <= delta, 0.5 * d * d, delta * (a - 0.5 * delta))
    n = max(float(mask.sum()), 1.0)
    g = np.where(a <= delta, d, delta * np.sign(d)) / n
    return float(loss_el.sum() / n), g


def backward(params, acts, pre, gy, emulate_bf16: bool = True):
    """Gradients of sum(gy * y) w.r.t. every W and b.

    The GPU multiplies bf16 copies of the weights and activations and the
    gradient of the layer output rounded to bf16; the same roundings are
    applied here when emulate_bf16 is set."""
    q = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    grads = [None] * len(params)
    g = np.asarray(gy, dtype=np.float64)
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        gq = q(g)
        gW = gq.T @ acts[i]
        gb = gq.sum(axis=0)
        grads[i] = (gW, gb)
        if i > 0:
            gh = gq @ q(W)
            g = gh * (pre[i - 1] > 0)
    return grads


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on FP64 copies; returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        res = []
        for p_, g_, m_, v_ in ((W, gW, mW, vW), (b, gb, mb, vb)):
            m2 = b1 * m_ + (1 - b1) * g_
            v2 = b2 * v_ + (1 - b2) * g_ * g_
            mh = m2 / (1 - b1 ** t)
            vh = v2 / (1 - b2 ** t)
            res.append((p_ - lr * mh / (np.sqrt(vh) + eps), m2, v2))
        out_p.append((res[0][0], res[1][0]))
        out_m.append((res[0][1], res[1][1]))
        out_v.append((res[0][2], res[1][2]))
    return out_p, out_m, out_v


def combo_cards():
    out = np.zeros((NCOMBO, 2), dtype=np.int64)
    for a in range(1, 52):
        for b in range(a):
            out[a * (a - 1) // 2 + b] = (a, b)
    return out


_CC = combo_cards()


def leaf_inputs(reach_leaf: np.ndarray, board, pot: float, stack_behind: float, d_in: int):
    """Network inputs of one depth-limit leaf for every next card.

    reach_leaf: [2, 1326] reach of both players at the leaf.  For each card c
    not on the board (ascending), the row holds each player's reach with the
    combos holding c removed, normalised to sum 1 (all zero if nothing is
    left), then a one-hot of the board plus c (52 entries), then the
    stack-to-pot ratio; zero padding up to d_in.  Returns (cards, X)."""
    cards = [c for c in range(52) if c not in board]
    X = np.zeros((len(cards), d_in), dtype=np.float64)
    for k, c in enumerate(cards):
        keep = (_CC[:, 0] != c) & (_CC[:, 1] != c)
        for p in range(2):
            v = reach_leaf[p] * keep
            s = v.sum()
            if s > 0:
                X[k, p * NCOMBO:(p + 1) * NCOMBO] = v / s
        for b in list(board) + [c]:
            X[k, 2 * NCOMBO + b] = 1.0
        X[k, 2 * NCOMBO + 52] = stack_behind / pot
    return cards, X


def _flop_keep(flops) -> np.ndarray:
    """[k, 1326] bool: combos holding no card of each flop."""
    flops = np.asarray(flops)
    keep = np.ones((len(flops), NCOMBO), dtype=bool)
    for j in range(3):
        c = flops[:, j][:, None]
        keep &= (_CC[:, 0][None, :] != c) & (_CC[:, 1][None, :] != c)
    return keep


def flop_leaf_inputs(reach_leaf: np.ndarray, flops, pot: float, stack_behind: float, d_in: int):
    """Network inputs of one preflop leaf for each flop of `flops` ([k, 3]
    cards): each player's reach with the combos holding a flop card removed,
    normalised to sum 1 (all zero if nothing is left), the flop's three cards
    one-hot (52 entries), the stack-to-pot ratio; zero padding up to d_in."""
    flops = np.asarray(flops)
    keep = _flop_keep(flops)
    X = np.zeros((len(flops), d_in), dtype=np.float64)
    for p in range(2):
        v = reach_leaf[p][None, :] * keep
        s = v.sum(axis=1)
        nz = s > 0
        X[nz, p * NCOMBO:(p + 1) * NCOMBO] = v[nz] / s[nz, None]
    rows = np.arange(len(flops))
    for j in range(3):
        X[rows, 2 * NCOMBO + flops[:, j]] = 1.0
    X[:, 2 * NCOMBO + 52] = stack_behind / pot
    return X


def flop_zero_sum_shifts(ev_rows: np.ndarray, reach_leaf: np.ndarray, flops) -> np.ndarray:
    """The zero-sum correction (as zero_sum_shift) of each row of a preflop
    leaf: ev_rows [k, 2, 1326] after flop flops[k]; only combos clear of the
    flop count, and M is the opponent reach clear of the hand and the flop
    (brute force over opponent combos, one product per player)."""
    keep = _flop_keep(flops)
    K = _compat()
    r0 = reach_leaf[0][None, :] * keep
    r1 = reach_leaf[1][None, :] * keep
    m1 = r1 @ K          # K is symmetric
    m0 = r0 @ K
    e = (r0 * m1 * ev_rows[:, 0]).sum(axis=1) + (r1 * m0 * ev_rows[:, 1]).sum(axis=1)
    z = (r0 * m1).sum(axis=1)
    out = np.zeros(len(keep))
    pos = z > 0
    out[pos] = e[pos] / (2.0 * z[pos])
    return out


_COMPAT = None


def _compat():
    """[1326, 1326] float64: 1 where two combos share no card."""
    global _COMPAT
    if _COMPAT is None:
        a, b = _CC[:, 0], _CC[:, 1]
        share = (a[:, None] == a[None, :]) | (a[:, None] == b[None, :]) | (b[:, None] == a[None, :]) | \
                (b[:, None] == b[None, :])
        _COMPAT = (~share).astype(np.float64)
    return _COMPAT


def compatible_mass(r_opp: np.ndarray, card: int) -> np.ndarray:
    """M(h | c) for every combo h: the opponent reach summed over combos that
    share no card with h and do not hold the dealt card c (brute force)."""
    keep = (_CC[:, 0] != card) & (_CC[:, 1] != card)
    return _compat() @ (r_opp * keep)


def zero_sum_shift(ev: np.ndarray, reach_leaf: np.ndarray, card: int) -> float:
    """The zero-sum correction of one leaf row (a reading; the paper does not
    say how leaf values are kept consistent).  ev: [2, 1326] network outputs
    (value per pot unit and per unit of compatible opponent reach) after the
    next card c; reach_leaf: [2, 1326].  Returns d such that subtracting d
    from both players' EVs makes sum_h r0 M1 EV0 + sum_h r1 M0 EV1 = 0, with
    only combos not holding c counted: d = e / (2 z), z = sum_h r0 M1."""
    keep = (_CC[:, 0] != card) & (_CC[:, 1] != card)
    r0, r1 = reach_leaf[0] * keep, reach_leaf[1] * keep
    m1 = compatible_mass(reach_leaf[1], card)
    m0 = compatible_mass(reach_leaf[0], card)
    e = float((r0 * m1 * ev[0]).sum() + (r1 * m0 * ev[1]).sum())
    z = float((r0 * m1).sum())
    return e / (2.0 * z) if z > 0 else 0.0


def zero_sum_shifts(ev_rows: np.ndarray, reach_leaf: np.ndarray, cards) -> np.ndarray:
    """zero_sum_shift for several next cards of one leaf at once: ev_rows
    [k, 2, 1326] (row j after next card cards[j]), reach_leaf [2, 1326];
    returns the k shifts.  The same sums as zero_sum_shift, with the
    compatible masses of all k cards formed by one product per player."""
    cards = np.asarray(cards)
    keep = (_CC[:, 0][None, :] != cards[:, None]) & (_CC[:, 1][None, :] != cards[:, None])   # [k, 1326]
    r0 = reach_leaf[0][None, :] * keep
    r1 = reach_leaf[1][None, :] * keep
    K = _compat()
    m1 = r1 @ K          # [k, 1326]: M over player 1's reach without the card (K is symmetric)
    m0 = r0 @ K
    e = (r0 * m1 * ev_rows[:, 0]).sum(axis=1) + (r1 * m0 * ev_rows[:, 1]).sum(axis=1)
    z = (r0 * m1).sum(axis=1)
    out = np.zeros(len(cards))
    pos = z > 0
    out[pos] = e[pos] / (2.0 * z[pos])
    return out
