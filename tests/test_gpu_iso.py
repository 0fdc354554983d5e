"""Suit isomorphism on the GPU: with suit-symmetric ranges the solver sweeps
one chance child per orbit and must reach the plain FP64 oracle's results
(which knows nothing of symmetry) to the FP64 bound, and the GPU's own
non-isomorphic solve up to rounding order."""
import numpy as np
import pytest

import oracle as O
from paper_2605_19928_amd import inputs as I
from paper_2605_19928_amd import pcfr as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def spec_of(board, stacks=(150, 150), sizes=(50,), max_raises=2):
    return dict(board=list(board), pot=100, stacks=stacks, sizes=list(sizes), allin=True, max_raises=max_raises,
                depth_limit=0)


@pytest.mark.parametrize("board,seed", [([50, 46, 26, 10], 1), ([48, 44, 21, 17], 2)])
def test_turn_iso_matches_oracle(board, seed):
    spec = spec_of(board)
    rng = np.random.default_rng(seed)
    r = np.stack([I.symmetric_range(rng, board, support=40), I.symmetric_range(rng, board, support=40)])
    T = 30
    say(f"case: suit-isomorphic turn board={board} seed={seed} T={T} support 40 orbits")
    gt = P.Tree(**spec)
    gi = P.Solver(gt, r, P.SolverConfig(dtype="f64", suit_iso=1))
    gp = P.Solver(gt, r, P.SolverConfig(dtype="f64"))
    say(f"  swept nodes: {gi.swept_nodes()} with isomorphism, {gp.swept_nodes()} without")
    assert gi.swept_nodes() < gp.swept_nodes()
    gi.iterate(T)
    gp.iterate(T)
    ot = O.Tree.holdem(**spec)
    os_ = O.Solver(ot, r, support_only=True)
    os_.iterate(T)
    pot = spec["pot"]
    mask = (r > 0) & ~I.blocked_mask(board)[None, :]
    for which in ("current", "avg"):
        d = np.abs(gi.root_cfv(which) - os_.root_cfv(which))[mask].max() / pot
        dp = np.abs(gi.root_cfv(which) - gp.root_cfv(which))[mask].max() / pot
        say(f"  root cfv ({which}) vs oracle {d:.3e} pot, vs non-isomorphic GPU {dp:.3e} pot")
        assert d <= 1e-9 and dp <= 1e-12
    eg, _ = gi.exploitability()
    eo, _ = os_.exploitability()
    say(f"  exploitability gpu {eg:.9f} oracle {eo:.9f} chips")
    assert abs(eg - eo) / pot <= 1e-9
    # strategies at every decision node: swept ones directly, skipped ones
    # through their representative with the hands relabelled
    m = gt.suit_iso_map(r)
    e = ot.export()
    worst = {False: 0.0, True: 0.0}
    for n in np.flatnonzero(e["type"] == O.T_DEC):
        own = mask[int(e["player"][n])]
        for which in ("avg", "current"):
            d = float(np.abs(gi.strategy(int(n), which) - os_.strategy(int(n), which))[:, own].max())
            worst[bool(m["skip"][n])] = max(worst[bool(m["skip"][n])], d)
    say(f"  strategies max |d|: swept nodes {worst[False]:.3e}, skipped nodes {worst[True]:.3e}")
    assert worst[False] <= 1e-9 and worst[True] <= 1e-9


def test_iso_without_symmetry_is_bitwise_plain():
    board = [50, 46, 26, 10]
    spec = spec_of(board)
    rng = np.random.default_rng(3)
    r = np.stack([I.dirichlet_range(rng, board, support=60), I.dirichlet_range(rng, board, support=60)])
    say(f"case: suit isomorphism on, ranges without symmetry, board={board}")
    gt = P.Tree(**spec)
    a = P.Solver(gt, r, P.SolverConfig(dtype="f32", suit_iso=1))
    b = P.Solver(gt, r, P.SolverConfig(dtype="f32"))
    assert a.swept_nodes() == b.swept_nodes()
    a.iterate(20)
    b.iterate(20)
    assert np.array_equal(a.root_cfv("avg"), b.root_cfv("avg"))


def test_batch_iso_matches_single_plain_solves():
    boards = [[50, 46, 26, 10], [48, 44, 21, 17], [51, 30, 13, 0]]
    rng = np.random.default_rng(4)
    specs, rs = [], []
    for i, b in enumerate(boards):
        specs.append(spec_of(b))
        if i < 2:
            rs.append(np.stack([I.symmetric_range(rng, b), I.symmetric_range(rng, b)]))
        else:
            rs.append(np.stack([I.dirichlet_range(rng, b), I.dirichlet_range(rng, b)]))
    say(f"case: batch of {len(boards)} turns (2 symmetric, 1 not) with suit isomorphism vs single plain solves, f64")
    trees = [P.Tree(**s) for s in specs]
    bt = P.Batch(trees, np.stack(rs), P.SolverConfig(dtype="f64", suit_iso=1))
    bt.iterate(15)
    for g in range(len(boards)):
        s = P.Solver(trees[g], rs[g], P.SolverConfig(dtype="f64"))
        s.iterate(15)
        d = np.abs(bt.root_cfv_of(g, "avg") - s.root_cfv("avg")).max() / 100
        say(f"  subgame {g}: root cfv (avg) max |d| = {d:.3e} pot")
        assert d <= 1e-12
        s.close()


def test_iso_on_unevenly_pruned_tree_matches_oracle():
    """Suit isomorphism on a tree pruned in one chance child's subtree only:
    the map pairs only subtrees of identical shape, so the isomorphic solve
    still equals the oracle's solve of the same reduced game."""
    board = [50, 46, 26, 10]
    spec = spec_of(board)
    rng = np.random.default_rng(4)
    r = np.stack([I.symmetric_range(rng, board, support=40), I.symmetric_range(rng, board, support=40)])
    T = 20
    say(f"case: suit isomorphism on an unevenly pruned turn, board={board} T={T}")
    gt, ot = P.Tree(**spec), O.Tree.holdem(**spec)
    m0 = gt.suit_iso_map(r)
    e = gt.export()
    node = int(np.flatnonzero(m0["perm"] >= 0)[0])
    while not (e["type"][node] == P.NODE_DECISION and e["n_child"][node] >= 2):
        node = int(e["first_child"][node])
    flags = np.zeros(gt.n_nodes, dtype=np.uint8)
    flags[int(e["first_child"][node]) + int(e["n_child"][node]) - 1] = 1
    gr, _ = gt.prune(flags)
    orr, _ = ot.prune(flags)
    gi = P.Solver(gr, r, P.SolverConfig(dtype="f64", suit_iso=1))
    gp = P.Solver(gr, r, P.SolverConfig(dtype="f64"))
    say(f"  swept nodes: {gi.swept_nodes()} with isomorphism, {gp.swept_nodes()} without")
    assert gi.swept_nodes() < gp.swept_nodes()
    gi.iterate(T)
    gp.iterate(T)
    os_ = O.Solver(orr, r, support_only=True)
    os_.iterate(T)
    pot = spec["pot"]
    mask = (r > 0) & ~I.blocked_mask(board)[None, :]
    for which in ("current", "avg"):
        d = np.abs(gi.root_cfv(which) - os_.root_cfv(which))[mask].max() / pot
        dp = np.abs(gi.root_cfv(which) - gp.root_cfv(which))[mask].max() / pot
        say(f"  root cfv ({which}) vs oracle {d:.3e} pot, vs non-isomorphic GPU {dp:.3e} pot")
        assert d <= 1e-9 and dp <= 1e-12
