"""Host-side checks of the HIP library (no GPU needed).

* The shared object loads and exports every function ``include/pcfr.h``
  declares.
* The library's tree builder (breadth-first queue) and the oracle's
  (depth-first, then renumbered) emit bit-identical node arrays.
* The library's bitmask evaluator and the oracle's best-of-21 evaluator agree
  on every tested seven-card hand.
* Invalid specs are rejected with PCFR_E_INVALID_ARG.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2605_19928_amd import inputs as I
from paper_2605_19928_amd import pcfr as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "pcfr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pcfr_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(P.LIB_PATH)
    names = header_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n
    assert L.pcfr_abi_version() == 2


SPECS = [
    I.river_config(0)[0],
    I.river_config(1)[0],
    I.turn_config(0, spr=1, pot=100)[0],
    I.turn_config(3, spr=2)[0],
    I.turn_config(4)[0],
    I.flop_config(0)[0],
    dict(board=[1, 9, 17], pot=40, stacks=(30, 500), sizes=[50], allin=True, max_raises=2, depth_limit=0),
    dict(board=[0, 4, 8, 12, 16], pot=2, stacks=(0, 0), sizes=[], allin=False, max_raises=0, depth_limit=0),
    # preflop roots: leaves at the flop deal, no all-in
    dict(board=[], pot=20, stacks=(1000, 1000), sizes=[100], allin=False, max_raises=1, depth_limit=1),
    dict(board=[], pot=20, stacks=(1000, 1000), sizes=[50, 100], allin=False, max_raises=3, depth_limit=1),
]


@pytest.mark.parametrize("spec", SPECS, ids=[f"s{i}" for i in range(len(SPECS))])
def test_tree_arrays_identical(spec):
    a = P.Tree(**spec)
    b = O.Tree.holdem(**spec)
    ea, eb = a.export(), b.export()
    assert a.n_nodes == b.n_nodes
    for k in ("type", "player", "parent", "action", "depth", "chance_card", "first_child", "n_child", "contrib"):
        np.testing.assert_array_equal(ea[k], eb[k], err_msg=k)
    assert (a.n_decision, a.n_fold, a.n_showdown, a.n_chance, a.n_leaf, a.n_allin, a.n_levels, a.n_rows) == \
        (b.n_decision, b.n_fold, b.n_showdown, b.n_chance, b.n_leaf, b.n_allin, b.n_levels, b.n_rows)
    nb = len(spec["board"])
    assert a.n_hands == {0: 169, 3: 1176, 4: 1128, 5: 1081}[nb]
    assert a.n_hands_padded % 64 == 0 and a.n_hands_padded >= a.n_hands


def test_evaluators_agree_on_random_hands():
    rng = np.random.default_rng(1)
    n = 400_000
    hands = np.argsort(rng.random((n, 52)), axis=1)[:, :7].astype(np.int32)
    np.testing.assert_array_equal(P.eval7_batch(hands), O.eval7_batch(hands))


def test_evaluators_agree_on_structured_hands():
    # every rank multiset pattern with flush-heavy suits
    rng = np.random.default_rng(2)
    rows = []
    for _ in range(50_000):
        suit = rng.integers(0, 4)
        k = rng.integers(3, 8)
        ranks = rng.choice(13, k, replace=False)
        cards = [4 * r + suit for r in ranks]
        while len(cards) < 7:
            c = int(rng.integers(0, 52))
            if c not in cards:
                cards.append(c)
        rows.append(cards[:7])
    hands = np.array(rows, dtype=np.int32)
    np.testing.assert_array_equal(P.eval7_batch(hands), O.eval7_batch(hands))


@pytest.mark.parametrize("bad", [
    dict(board=[0, 1], pot=100, stacks=(400, 400), sizes=[50]),
    dict(board=[0, 1, 1], pot=100, stacks=(400, 400), sizes=[50]),
    dict(board=[0, 1, 52], pot=100, stacks=(400, 400), sizes=[50]),
    dict(board=[0, 1, 2], pot=101, stacks=(400, 400), sizes=[50]),
    dict(board=[0, 1, 2], pot=100, stacks=(-1, 400), sizes=[50]),
    dict(board=[0, 1, 2], pot=100, stacks=(400, 400), sizes=[75, 50]),
    dict(board=[0, 1, 2], pot=100, stacks=(400, 400), sizes=[0]),
])
def test_invalid_specs_rejected(bad):
    with pytest.raises(P.PcfrError) as e:
        P.Tree(**bad)
    assert e.value.code == P.E_INVALID_ARG


@pytest.mark.parametrize("bad", [
    dict(board=[], pot=20, stacks=(1000, 1000), sizes=[100], allin=False, max_raises=1, depth_limit=0),
    dict(board=[], pot=20, stacks=(1000, 1000), sizes=[100], allin=True, max_raises=1, depth_limit=1),
    dict(board=[], pot=20, stacks=(15, 15), sizes=[100], allin=False, max_raises=1, depth_limit=1),
])
def test_unsupported_preflop_specs_refused(bad):
    """A preflop root must stop at the flop and never put a player all in;
    the oracle refuses the same specs."""
    with pytest.raises(P.PcfrError) as e:
        P.Tree(**bad)
    assert e.value.code == P.E_UNSUPPORTED
    with pytest.raises(ValueError):
        O.Tree.holdem(**bad)


@pytest.mark.parametrize("nb", [4, 3])
def test_equity_table_matches_oracle(nb):
    rng = np.random.default_rng(20 + nb)
    board = I.draw_board(rng, nb)
    spec = dict(board=board, pot=100, stacks=(400, 400), sizes=[75], allin=True, max_raises=1, depth_limit=1)
    lib_t = P.Tree(**spec)
    ora_t = O.Tree.holdem(**spec)
    leaf = int(np.flatnonzero(ora_t.export()["type"] == O.T_LEAF)[0])
    np.testing.assert_array_equal(lib_t.equity_table(), ora_t.equity_table(leaf))


@pytest.mark.parametrize("spec", SPECS[:6], ids=[f"s{i}" for i in range(6)])
def test_pruned_tree_arrays_identical(spec):
    """The library's reduced tree of online pruning (one pass over the
    breadth-first ids) against the oracle's (a rebuilt pool renumbered
    breadth-first), for the same random flags."""
    a = P.Tree(**spec)
    b = O.Tree.holdem(**spec)
    e = a.export()
    rng = np.random.default_rng(len(e["type"]))
    flags = np.zeros(a.n_nodes, dtype=np.uint8)
    for n in np.flatnonzero(e["type"] == P.NODE_DECISION):
        fc, A = int(e["first_child"][n]), int(e["n_child"][n])
        if A >= 2 and rng.random() < 0.3:
            flags[fc + rng.integers(A)] = 1
    ra, ma = a.prune(flags)
    rb, mb = b.prune(flags)
    assert ra.n_nodes == rb.n_nodes < a.n_nodes
    np.testing.assert_array_equal(ma, mb)
    ea, eb = ra.export(), rb.export()
    for k in ("type", "player", "parent", "action", "depth", "chance_card", "first_child", "n_child", "contrib"):
        np.testing.assert_array_equal(ea[k], eb[k], err_msg=k)
    assert (ra.n_decision, ra.n_fold, ra.n_showdown, ra.n_chance, ra.n_leaf, ra.n_allin, ra.n_levels, ra.n_rows) == \
        (rb.n_decision, rb.n_fold, rb.n_showdown, rb.n_chance, rb.n_leaf, rb.n_allin, rb.n_levels, rb.n_rows)


def test_prune_rejects_invalid_flags():
    a = P.Tree(**SPECS[0])
    e = a.export()
    flags = np.zeros(a.n_nodes, dtype=np.uint8)
    flags[0] = 1
    with pytest.raises(P.PcfrError):
        a.prune(flags)
    flags[:] = 0
    n = int(np.flatnonzero(e["type"] == P.NODE_DECISION)[0])
    flags[e["first_child"][n]: e["first_child"][n] + e["n_child"][n]] = 1
    with pytest.raises(P.PcfrError):
        a.prune(flags)


def _batch_workspace(trees):
    cfg = P.SolverConfig().to_c()
    arr = (ctypes.c_void_p * len(trees))(*[t._h.value for t in trees])
    nb = ctypes.c_size_t()
    rc = P.lib().pcfr_batch_workspace_bytes(arr, len(trees), ctypes.byref(cfg), ctypes.byref(nb))
    return rc, int(nb.value)


def test_batch_of_depth_limited_subgames_planned():
    """Depth-limited subgames batch when every subgame holding leaves has a
    board of one size (a river without leaves may join); a flop and a
    depth-limited turn together are refused."""
    flops = [P.Tree(**I.flop_config(s, support=150)[0]) for s in (0, 2)]
    river = P.Tree(board=[0, 13, 26, 39, 51], pot=100, stacks=(400, 400), sizes=[75], allin=True, max_raises=1)
    rc, nb = _batch_workspace([river] + flops)
    assert rc == P.OK and nb > 0
    rc1, nb1 = _batch_workspace(flops[:1])
    assert rc1 == P.OK and nb1 < nb
    turn = P.Tree(board=[0, 13, 26, 40], pot=100, stacks=(400, 400), sizes=[75], allin=True, max_raises=1,
                  depth_limit=1)
    assert turn.n_leaf > 0
    rc, _ = _batch_workspace([flops[0], turn])
    assert rc == P.E_UNSUPPORTED
    assert "one size" in P.lib().pcfr_last_error().decode()


def test_empty_batch_refused_before_any_device_call():
    """A batch of no subgames has no plan: sizing and creation both return
    PCFR_E_INVALID_ARG (checked before anything touches a device)."""
    cfg = P.SolverConfig().to_c()
    nb = ctypes.c_size_t(123)
    arr = (ctypes.c_void_p * 1)(P.Tree(**SPECS[0])._h.value)
    L = P.lib()
    assert L.pcfr_batch_workspace_bytes(arr, 0, ctypes.byref(cfg), ctypes.byref(nb)) == 1
    ranges = np.zeros(2 * 1326)
    buf = ctypes.create_string_buffer(512)
    ws = (ctypes.addressof(buf) + 255) // 256 * 256
    out = ctypes.c_void_p()
    rc = L.pcfr_batch_create(arr, 0, ctypes.byref(cfg), ranges.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(ws),
                             ctypes.c_size_t(256), None, ctypes.byref(out))
    assert rc == 1 and not out.value
