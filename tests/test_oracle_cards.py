"""Pins for the oracle's hand evaluator against published hand-category counts.

The counts of five-card and seven-card poker hands by category are textbook
values (e.g. the standard combinatorics tables for a 52-card deck); the number
of distinct five-card equivalence classes is 7462.
"""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_2605_19928_amd import inputs as I

# high, pair, two pair, trips, straight, flush, full house, quads, straight flush
C5 = [1302540, 1098240, 123552, 54912, 10200, 5108, 3744, 624, 40]
C7 = [23294460, 58627800, 31433400, 6461620, 6180020, 4047644, 3473184, 224848, 41584]


def card(s):
    r = "23456789TJQKA".index(s[0])
    u = "cdhs".index(s[1])
    return 4 * r + u


def ev(*cs):
    cards = [card(c) for c in cs]
    return O.eval5(cards) if len(cards) == 5 else O.eval7(cards)


def test_five_card_category_counts():
    assert list(O.category_counts(5)) == C5


def test_distinct_five_card_classes():
    assert O.distinct5() == 7462


@pytest.mark.slow
def test_seven_card_category_counts():
    assert list(O.category_counts(7)) == C7


def test_encoding_examples():
    # category in bits 20..23, tie-break ranks below
    assert ev("As", "Ks", "Qs", "Js", "Ts") == (8 << 20) | (12 << 16)
    assert ev("5d", "4d", "3d", "2d", "Ad") == (8 << 20) | (3 << 16)       # steel wheel: high card 5
    assert ev("5d", "4c", "3d", "2d", "Ad") == (4 << 20) | (3 << 16)       # wheel
    assert ev("6d", "5c", "4d", "3d", "2h") > ev("5d", "4c", "3d", "2d", "Ad")
    assert ev("Kh", "Kd", "Kc", "2s", "2d") > ev("Qh", "Qd", "Qc", "As", "Ad")
    assert ev("Ah", "Ad", "Kc", "Ks", "2d") > ev("Ah", "Ad", "Qc", "Qs", "Kd")
    assert ev("Ah", "Ad", "Kc", "Ks", "3d") > ev("Ah", "Ad", "Kc", "Ks", "2d")
    assert ev("2h", "2d", "2c", "2s", "3d") == (7 << 20) | (0 << 16) | (1 << 12)
    # seven cards: best five
    assert ev("As", "Ks", "Qs", "Js", "Ts", "2d", "2c") == (8 << 20) | (12 << 16)
    assert ev("Ah", "Ad", "Ac", "Kd", "Kc", "Qh", "Qd") == (6 << 20) | (12 << 16) | (11 << 12)
    assert ev("7h", "6d", "5c", "4d", "3c", "2h", "Ad") == (4 << 20) | (5 << 16)


def test_seven_is_max_of_fives_on_random_hands():
    rng = np.random.default_rng(7)
    hands = np.stack([rng.choice(52, 7, replace=False) for _ in range(300)]).astype(np.int32)
    got = O.eval7_batch(hands)
    for h, v in zip(hands, got):
        best = max(O.eval5(list(s)) for s in itertools.combinations(h, 5))
        assert v == best


def test_combo_index_bijection():
    cc = I.combo_cards()
    seen = set()
    for k, (a, b) in enumerate(cc):
        assert a > b and a * (a - 1) // 2 + b == k
        seen.add((int(a), int(b)))
    assert len(seen) == 1326
