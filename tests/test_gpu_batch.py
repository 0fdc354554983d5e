"""Batched subgames: one forest advanced by the same launches.

Every subgame of a batch must come out bitwise identical to solving it alone
(the kernels do the same arithmetic per node and hand; padding lanes add
exact zeros), and a sampled subgame of the batch is checked against the
oracle.  Sizes are uneven: rivers and turns with 1-4 bet sizes.
"""
import numpy as np
import pytest

import oracle as O
from paper_2605_19928_amd import inputs as I
from paper_2605_19928_amd import pcfr as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def count_nodes(spec):
    return P.Tree(**spec).n_nodes


def test_batched_equals_individual_bitwise():
    cases = I.batch_config(3, count_nodes, n=8, river_share=0.6, lo=10, hi=900)
    say("case: batch sizes", [count_nodes(s) for s, _ in cases])
    trees = [P.Tree(**s) for s, _ in cases]
    ranges = np.stack([r for _, r in cases])
    b = P.Batch(trees, ranges)
    T = 25
    b.iterate(T)
    eb, brb = b.exploitability_all()
    for g, (spec, r) in enumerate(cases):
        s = P.Solver(trees[g], r)
        s.iterate(T)
        np.testing.assert_array_equal(b.root_cfv_of(g, "current"), s.root_cfv("current"))
        e = trees[g].export()
        for n in np.flatnonzero(e["type"] == P.NODE_DECISION)[:6]:
            np.testing.assert_array_equal(b.strategy_of(g, int(n)), s.strategy(int(n)))
        es, brs = s.exploitability()
        assert es == eb[g] and np.array_equal(brs, brb[g])
        s.close()


def test_batch_member_matches_oracle():
    cases = I.batch_config(4, count_nodes, n=6, river_share=0.5, lo=10, hi=600)
    trees = [P.Tree(**s) for s, _ in cases]
    ranges = np.stack([r for _, r in cases])
    b = P.Batch(trees, ranges, P.SolverConfig(dtype="f64"))
    T = 15
    b.iterate(T)
    e_all, _ = b.exploitability_all()
    for g in (0, 2):                      # river members: the oracle runs them at full ranges
        spec, r = cases[g]
        say(f"case: batch member {g} {spec}")
        ot = O.Tree.holdem(**spec)
        os_ = O.Solver(ot, r)
        os_.iterate(T)
        d = np.abs(b.root_cfv_of(g, "current") - os_.root_cfv("current")).max() / spec["pot"]
        eo, _ = os_.exploitability()
        say(f"  root cfv max |d| = {d:.3e} pot; exploitability batch {e_all[g]:.9f} oracle {eo:.9f}")
        assert d <= 1e-9 and abs(e_all[g] - eo) / spec["pot"] <= 1e-9


def test_autotune_keeps_iterates_bitwise():
    """The autotuner only changes workgroup sizes: a tuned batch must iterate
    bitwise like one created before tuning, and tuning leaves t = 0."""
    cases = I.batch_config(5, count_nodes, n=12, river_share=0.7, lo=10, hi=1500)
    trees = [P.Tree(**s) for s, _ in cases]
    ranges = np.stack([r for _, r in cases])
    ref = P.Batch(trees, ranges)           # schedule fixed at creation, before any tuning below
    tuned = P.Batch(trees, ranges)
    before, after = tuned.autotune(2)
    say(f"case: autotune 12 subgames, {before:.4f} -> {after:.4f} ms/iter")
    assert before > 0 and after > 0 and tuned.t == 0
    T = 20
    ref.iterate(T)
    tuned.iterate(T)
    for g in range(len(cases)):
        np.testing.assert_array_equal(tuned.root_cfv_of(g, "current"), ref.root_cfv_of(g, "current"))
        e = trees[g].export()
        for n in np.flatnonzero(e["type"] == P.NODE_DECISION)[:4]:
            np.testing.assert_array_equal(tuned.strategy_of(g, int(n)), ref.strategy_of(g, int(n)))
    with pytest.raises(P.PcfrError):
        tuned.autotune(1)                  # only a solver that has not iterated can be tuned


def test_autotune_with_budget():
    cases = I.batch_config(7, count_nodes, n=6, river_share=1.0, lo=10, hi=2000)
    trees = [P.Tree(**s) for s, _ in cases]
    b = P.Batch(trees, np.stack([r for _, r in cases]))
    b.autotune_budget(50)
    assert b.t == 0
    b.iterate(3)
    assert b.t == 3


def depth_limited_cases():
    """A river (no leaves) first, then two depth-limited flops on different
    boards: subgame 0 has no leaves and another board size, so every leaf
    table is read at a subgame index other than 0."""
    river = I.batch_config(6, count_nodes, n=1, river_share=1.0, lo=10, hi=300)[0]
    flops = [I.flop_config(s, support=150) for s in (0, 2)]
    return [river] + flops


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_depth_limited_exact_leaves(dtype):
    cases = depth_limited_cases()
    say(f"case: batch of a river and two depth-limited flops, exact leaves, {dtype}")
    trees = [P.Tree(**s) for s, _ in cases]
    assert [t.n_leaf > 0 for t in trees] == [False, True, True]
    b = P.Batch(trees, np.stack([r for _, r in cases]), P.SolverConfig(dtype=dtype))
    T = 12
    b.iterate(T)
    eb, _ = b.exploitability_all()
    for g, (spec, r) in enumerate(cases):
        s = P.Solver(trees[g], r, P.SolverConfig(dtype=dtype))
        s.iterate(T)
        np.testing.assert_array_equal(b.root_cfv_of(g, "current"), s.root_cfv("current"))
        np.testing.assert_array_equal(b.root_cfv_of(g, "avg"), s.root_cfv("avg"))
        es, _ = s.exploitability()
        assert es == eb[g]
        s.close()
    if dtype == "f64":
        spec, r = cases[2]
        ot = O.Tree.holdem(**spec)
        os_ = O.Solver(ot, r)
        os_.iterate(T)
        ok = ~I.blocked_mask(spec["board"])
        d = np.abs(b.root_cfv_of(2, "current") - os_.root_cfv("current"))[:, ok].max() / spec["pot"]
        say(f"  member 2 against the oracle: root cfv max |d| = {d:.3e} pot")
        assert d <= 1e-9


@pytest.mark.parametrize("variant,alternating", [("pcfr+", 1), ("cfr+", 0)])
def test_batch_depth_limited_variants(variant, alternating):
    """The other update rules on a batch with exact leaves: members bitwise
    equal to their own solves (alternating updates sweep each player in turn,
    so the leaves are evaluated twice per iteration)."""
    cases = depth_limited_cases()
    say(f"case: batch of a river and two depth-limited flops, {variant}, alternating {alternating}")
    cfg = P.SolverConfig(dtype="f64", variant=variant, alternating=alternating)
    trees = [P.Tree(**s) for s, _ in cases]
    b = P.Batch(trees, np.stack([r for _, r in cases]), cfg)
    T = 8
    b.iterate(T)
    for g, (spec, r) in enumerate(cases):
        s = P.Solver(trees[g], r, cfg)
        s.iterate(T)
        np.testing.assert_array_equal(b.root_cfv_of(g, "current"), s.root_cfv("current"))
        e = trees[g].export()
        for n in np.flatnonzero(e["type"] == P.NODE_DECISION)[:4]:
            np.testing.assert_array_equal(b.strategy_of(g, int(n)), s.strategy(int(n)))
        s.close()


def depth_limited_turn_cases():
    """A river, then two depth-limited turns (leaves at the river card) on
    different 4-card boards."""
    river = I.batch_config(6, count_nodes, n=1, river_share=1.0, lo=10, hi=300)[0]
    out = [river]
    for seed in (3, 5):
        rng = np.random.default_rng(seed)
        board = I.draw_board(rng, 4)
        r = np.stack([I.dirichlet_range(rng, board, 1.0, 150), I.dirichlet_range(rng, board, 1.0, 150)])
        out.append((dict(board=board, pot=100, stacks=(400, 400), sizes=[50, 100], allin=True, max_raises=2,
                         depth_limit=1), r))
    return out


@pytest.mark.parametrize("street", ["flop", "turn"])
def test_batch_depth_limited_network_leaves(street):
    """With a leaf network, the batch feeds every subgame's (leaf, next card)
    rows through one set of GEMMs; on fixed tiles each member must match its
    own solve bitwise."""
    cases = depth_limited_cases() if street == "flop" else depth_limited_turn_cases()
    trees = [P.Tree(**s) for s, _ in cases]
    b = P.Batch(trees, np.stack([r for _, r in cases]), P.SolverConfig(dtype="f64"))
    n_leaves, n_next = b.leaf_rows()
    assert n_leaves == trees[1].n_leaf + trees[2].n_leaf and n_next == (49 if street == "flop" else 48)
    rng = np.random.default_rng(17)
    params = None

    def make_net(rows):
        nonlocal params
        net = P.LeafNet(P.LEAF_D_IN, 64, 2, P.LEAF_D_OUT, max_batch=rows)
        if params is None:
            params = [((rng.standard_normal((o, i)) * 2.0 / np.sqrt(i)).astype(np.float32),
                       (rng.standard_normal(o) * 0.05).astype(np.float32)) for o, i in net.layer_shapes()]
        net.set_params(params)
        net.tiles = [0] * len(params)
        return net

    # a network sized for one subgame's rows is refused by the batch
    small = make_net(trees[1].n_leaf * n_next)
    with pytest.raises(P.PcfrError, match="max_batch"):
        b.attach_leafnet(small)
    small.close()
    netb = make_net(n_leaves * n_next)
    b.attach_leafnet(netb)
    say(f"case: batch with a leaf network, {n_leaves} leaves x {n_next} next cards")
    T = 3
    b.iterate(T)
    for g in (1, 2):
        spec, r = cases[g]
        s = P.Solver(trees[g], r, P.SolverConfig(dtype="f64"))
        nl, nn = s.leaf_rows()
        net = make_net(nl * nn)
        s.attach_leafnet(net)
        s.iterate(T)
        d = np.abs(b.root_cfv_of(g, "current") - s.root_cfv("current")).max()
        say(f"  member {g}: root cfv max |d| against its own solve = {d:.3e}")
        np.testing.assert_array_equal(b.root_cfv_of(g, "current"), s.root_cfv("current"))
        s.close()


@pytest.mark.parametrize("dtype,variant", [("f32", "dcfr"), ("f64", "dcfr"), ("f32", "pcfr+")])
def test_persistent_launch_is_bitwise_the_graph(dtype, variant):
    """One cooperative launch running all iterations (grid barriers between
    the level sweeps and the terminals) against graph replays of per-level
    launches: the same iterates, bit for bit."""
    cases = I.batch_config(6, count_nodes, n=12, river_share=0.7, lo=10, hi=1500)
    trees = [P.Tree(**s) for s, _ in cases]
    ranges = np.stack([r for _, r in cases])
    say(f"case: persistent launch vs graph, 12 subgames, {dtype} {variant}")
    cfg = P.SolverConfig(dtype=dtype, variant=variant)
    g = P.Batch(trees, ranges, cfg)
    p = P.Batch(trees, ranges, cfg)
    p.set_launch(True)
    T = 20
    g.iterate(T)
    p.iterate(7)
    p.iterate(T - 7)
    assert p.t == g.t == T
    assert p.save_state() == g.save_state()
    for k in (0, 5, 11):
        np.testing.assert_array_equal(p.root_cfv_of(k, "current"), g.root_cfv_of(k, "current"))


def test_persistent_launch_refuses_what_it_does_not_run():
    spec, r = I.flop_config(0, support=100)
    s = P.Solver(P.Tree(**spec), r)
    with pytest.raises(P.PcfrError) as e:
        s.set_launch(True)
    assert e.value.code == P.E_UNSUPPORTED
    spec, r = I.river_config(2)
    s = P.Solver(P.Tree(**spec), r, P.SolverConfig(alternating=1))
    with pytest.raises(P.PcfrError):
        s.set_launch(True)


def test_batch_of_256_subgames():
    """The batching workload at its configured size: 256 river and turn
    subgames (70% rivers) of uneven trees in one forest, FP32.  The
    persistent launch and the graph give the same iterates bit for bit,
    sampled members equal their own solves bit for bit, and river members
    solved in FP64 match the oracle at 1e-9 pot."""
    cases = I.batch_config(0, count_nodes, n=256, river_share=0.7, lo=10, hi=2000)
    trees = [P.Tree(**s) for s, _ in cases]
    ranges = np.stack([r for _, r in cases])
    say(f"case: 256-subgame batch, {sum(t.n_nodes for t in trees)} nodes")
    T = 12
    g = P.Batch(trees, ranges)
    g.iterate(T)
    p = P.Batch(trees, ranges)
    p.set_launch(True)
    p.iterate(T)
    assert p.save_state() == g.save_state()
    del p
    rng = np.random.default_rng(1)
    for k in sorted(rng.choice(256, 6, replace=False)):
        s = P.Solver(trees[k], ranges[k])
        s.iterate(T)
        np.testing.assert_array_equal(g.root_cfv_of(int(k), "current"), s.root_cfv("current"))
        e = trees[k].export()
        n = int(np.flatnonzero(e["type"] == P.NODE_DECISION)[-1])
        np.testing.assert_array_equal(g.strategy_of(int(k), n), s.strategy(n))
        s.close()
    del g
    b = P.Batch(trees, ranges, P.SolverConfig(dtype="f64"))
    b.set_launch(True)
    b.iterate(T)
    e_all, _ = b.exploitability_all()
    rivers = [k for k, (sp, _) in enumerate(cases) if len(sp["board"]) == 5]
    for k in (rivers[0], rivers[len(rivers) // 2]):
        spec, r = cases[k]
        ot = O.Tree.holdem(**spec)
        os_ = O.Solver(ot, r)
        os_.iterate(T)
        d = np.abs(b.root_cfv_of(k, "current") - os_.root_cfv("current")).max() / spec["pot"]
        eo, _ = os_.exploitability()
        say(f"  member {k} ({ot.n_nodes} nodes): root cfv max |d| = {d:.3e} pot; exploitability batch "
            f"{e_all[k]:.9f} oracle {eo:.9f}")
        assert d <= 1e-9 and abs(e_all[k] - eo) / spec["pot"] <= 1e-9
