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
