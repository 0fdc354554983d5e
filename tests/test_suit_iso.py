"""Suit isomorphism map of the library (host side, no GPU) against a
brute-force reading of its definition: the group is every suit permutation
fixing the root board and both ranges; at each chance node outside skipped
subtrees, a child's orbit under the permutations that also fix the cards
dealt above the node is found by applying all of them, its representative is
the orbit's smallest card, and a mapped child's permutation carries the
representative's card to its own; skipped nodes are exactly the subtrees of
mapped children."""
import itertools

import numpy as np

from paper_2605_19928_amd import inputs as I
from paper_2605_19928_amd import pcfr as P

PERMS = list(itertools.permutations(range(4)))     # lexicographic, as the library's


def mapc(p, c):
    return 4 * (c // 4) + p[c % 4]


def combo(a, b):
    hi, lo = max(a, b), min(a, b)
    return hi * (hi - 1) // 2 + lo


def brute_group(board, r):
    cc = I.combo_cards()
    bits = 0
    for q, p in enumerate(PERMS):
        if {mapc(p, c) for c in board} != set(board):
            continue
        idx = np.array([combo(mapc(p, int(a)), mapc(p, int(b))) for a, b in cc])
        if np.array_equal(r[:, idx], r):
            bits |= 1 << q
    return bits


def check_map(spec, r):
    t = P.Tree(**spec)
    m = t.suit_iso_map(r)
    e = t.export()
    grp = brute_group(spec["board"], r)
    assert m["group"] == grp
    group = [q for q in range(24) if grp >> q & 1]
    n = t.n_nodes
    dealt = [frozenset()] * n
    for i in range(n):
        par = int(e["parent"][i])
        if par >= 0:
            c = int(e["chance_card"][i])
            dealt[i] = dealt[par] | ({c} if c >= 0 else set())
    skip = np.zeros(n, dtype=bool)
    for i in range(n):
        par = int(e["parent"][i])
        skip[i] = par >= 0 and (skip[par] or m["perm"][i] >= 0)
    assert np.array_equal(m["skip"].astype(bool), skip)
    is_chance_child = np.zeros(n, dtype=bool)
    for i in np.flatnonzero(e["type"] == P.NODE_CHANCE):
        kids = list(range(int(e["first_child"][i]), int(e["first_child"][i] + e["n_child"][i])))
        is_chance_child[kids] = True
        if skip[i]:
            continue
        gn = [q for q in group if {mapc(PERMS[q], c) for c in dealt[i]} == dealt[i]]
        card_child = {int(e["chance_card"][k]): k for k in kids}
        for k in kids:
            c = int(e["chance_card"][k])
            orbit = {mapc(PERMS[q], c) for q in gn} if len(gn) > 1 else {c}
            assert orbit <= set(card_child)
            rep = min(orbit)
            assert m["src"][k] == card_child[rep]
            if c == rep:
                assert m["perm"][k] == -1
            else:
                q = int(m["perm"][k])
                assert q in gn and mapc(PERMS[q], rep) == c
    others = ~is_chance_child
    assert (m["src"][others] == -1).all() and (m["perm"][others] == -1).all()
    return m, skip


def spec_of(board, depth_limit=0, stacks=(150, 150), sizes=(50,), max_raises=2):
    return dict(board=list(board), pot=100, stacks=stacks, sizes=list(sizes), allin=True, max_raises=max_raises,
                depth_limit=depth_limit)


def test_monotone_turn_uniform_ranges():
    board = [50, 46, 26, 10]                     # one suit: the other three are interchangeable
    r = np.where(I.blocked_mask(board), 0.0, 1.0)[None, :].repeat(2, axis=0)
    m, skip = check_map(spec_of(board), r)
    assert bin(m["group"]).count("1") == 6
    assert skip.sum() > 0


def test_two_suit_turn_symmetric_ranges():
    board = [48, 44, 21, 17]                     # suits {0, 0, 1, 1}: only suits 2 and 3 swap
    rng = np.random.default_rng(3)
    r = np.stack([I.symmetric_range(rng, board), I.symmetric_range(rng, board)])
    m, skip = check_map(spec_of(board), r)
    assert bin(m["group"]).count("1") == 2
    assert skip.sum() > 0


def test_asymmetric_ranges_map_nothing():
    board = [50, 46, 26, 10]
    rng = np.random.default_rng(4)
    r = np.stack([I.dirichlet_range(rng, board), I.dirichlet_range(rng, board)])
    m, skip = check_map(spec_of(board), r)
    assert m["group"] == 1 and skip.sum() == 0 and (m["perm"] < 0).all()


def test_one_symmetric_player_is_not_enough():
    board = [50, 46, 26, 10]
    rng = np.random.default_rng(5)
    r = np.stack([I.symmetric_range(rng, board), I.dirichlet_range(rng, board)])
    m, _ = check_map(spec_of(board), r)
    assert m["group"] == 1


def test_flop_to_showdown_nested_chance():
    board = [48, 44, 40]                          # monotone flop
    rng = np.random.default_rng(6)
    r = np.stack([I.symmetric_range(rng, board), I.symmetric_range(rng, board)])
    m, skip = check_map(spec_of(board, stacks=(100, 100), max_raises=1), r)
    assert bin(m["group"]).count("1") == 6 and skip.sum() > 0


def test_symmetric_range_is_invariant():
    board = [48, 44, 21, 17]
    rng = np.random.default_rng(7)
    r = I.symmetric_range(rng, board, support=30)
    cc = I.combo_cards()
    for p in I.suit_stabilizer(board):
        idx = np.array([combo(mapc(p, int(a)), mapc(p, int(b))) for a, b in cc])
        assert np.array_equal(r[idx], r)
    assert abs(r.sum() - 1.0) < 1e-12 and (r[I.blocked_mask(board)] == 0).all()


def _subtree_shape(e, root, perm):
    """Node-by-node shape of a subtree: types, action counts, players and
    contributions in action order, chance children keyed by their card (mapped
    through the suit permutation `perm`, identity when None)."""
    out = []
    stack = [root]
    while stack:
        v = stack.pop()
        out.append((int(e["type"][v]), int(e["n_child"][v]), int(e["player"][v]),
                    int(e["contrib"][v][0]), int(e["contrib"][v][1])))
        kids = list(range(int(e["first_child"][v]), int(e["first_child"][v]) + int(e["n_child"][v])))
        if e["type"][v] == P.NODE_CHANCE:
            key = (lambda c: mapc(perm, c)) if perm is not None else (lambda c: c)
            kids = sorted(kids, key=lambda x: key(int(e["chance_card"][x])))
        stack.extend(reversed(kids))
    return out


def test_unevenly_pruned_tree_maps_only_identical_subtrees():
    """A tree pruned in one chance child's subtree only: the suit permutations
    moving that child no longer map the game onto itself and leave the group;
    the child is paired with no other; every pair the map makes has identical
    subtrees."""
    board = [50, 46, 26, 10]
    spec = dict(board=board, pot=100, stacks=(150, 150), sizes=[50], allin=True, max_raises=2, depth_limit=0)
    rng = np.random.default_rng(4)
    r = np.stack([I.symmetric_range(rng, board, support=40), I.symmetric_range(rng, board, support=40)])
    t = P.Tree(**spec)
    m0 = t.suit_iso_map(r)
    e = t.export()
    # a mapped chance child, and the first decision with two or more actions in its subtree
    mapped = np.flatnonzero((m0["perm"] >= 0))
    assert len(mapped) > 0
    child = int(mapped[0])
    partner = int(m0["src"][child])
    node = child
    while not (e["type"][node] == P.NODE_DECISION and e["n_child"][node] >= 2):
        node = int(e["first_child"][node])
    flags = np.zeros(t.n_nodes, dtype=np.uint8)
    flags[int(e["first_child"][node]) + int(e["n_child"][node]) - 1] = 1
    tp, new = t.prune(flags)
    m = tp.suit_iso_map(r)
    f = tp.export()
    c, pa = int(new[child]), int(new[partner])
    assert m["src"][c] == c and m["perm"][c] < 0          # no longer read through its partner
    assert all(m["src"][x] != c for x in range(tp.n_nodes) if x != c)
    for x in np.flatnonzero(m["perm"] >= 0):
        s = int(m["src"][x])
        assert _subtree_shape(f, x, None) == _subtree_shape(f, s, PERMS[int(m["perm"][x])])
    # the symmetry group shrinks to the permutations that map the pruned tree
    # onto itself, and what survives still maps some children
    assert m["group"] != m0["group"] and (m["group"] & ~m0["group"]) == 0
    for q in range(24):
        if m["group"] >> q & 1:
            assert _subtree_shape(f, 0, PERMS[q]) == _subtree_shape(f, 0, None)
    assert (m["perm"] >= 0).sum() > 0
    assert pa >= 0
