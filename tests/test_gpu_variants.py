"""Stage-7 variants (CFR+, predictive CFR+) and alternating updates on the GPU vs the oracle.

The paper changes only the regret update between CFR variants (Sec. 4.4) and
compares DCFR with PCFR+ (Sec. 5, convergence).  FP64: 1e-9 pot on root
values, exploitability and every average and current strategy entry.
Checkpoints of PCFR+ carry the last instantaneous regret, so resuming from a
save is bitwise identical to running on.
"""
import numpy as np
import pytest

import oracle as O
from paper_2605_19928_amd import inputs as I
from paper_2605_19928_amd import pcfr as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("variant,alternating,which", [
    ("cfr+", False, "river"), ("pcfr+", False, "river"), ("dcfr", True, "river"), ("pcfr+", True, "river"),
    ("cfr+", False, "turn"), ("pcfr+", False, "turn")])
def test_variant_matches_oracle(variant, alternating, which):
    if which == "river":
        spec, r = I.river_config(4, support=140)
        so = False
    else:
        spec, r = I.turn_config(5, support=40, spr=1.5)
        so = True
    T = 40
    say(f"case: {variant} alternating={alternating} {which} {spec} T={T}")
    ot = O.Tree.holdem(**spec)
    os_ = O.Solver(ot, r, support_only=so, variant=variant, alternating=alternating)
    os_.iterate(T)
    gt = P.Tree(**spec)
    gs = P.Solver(gt, r, P.SolverConfig(dtype="f64", variant=variant, alternating=int(alternating)))
    gs.iterate(T)
    pot = spec["pot"]
    mask = (r > 0) if so else np.ones_like(r, dtype=bool)
    mask &= ~I.blocked_mask(spec["board"])[None, :]
    d = np.abs(gs.root_cfv("current") - os_.root_cfv("current"))[mask].max() / pot
    eg, _ = gs.exploitability()
    eo, _ = os_.exploitability()
    say(f"  root cfv max |d| = {d:.3e} pot, exploitability gpu {eg:.9f} oracle {eo:.9f}")
    assert d <= 1e-9 and abs(eg - eo) / pot <= 1e-9
    e = gt.export()
    for n in np.flatnonzero(e["type"] == P.NODE_DECISION):
        own = mask[int(e["player"][n])]
        for w in ("avg", "current"):
            diff = np.abs(gs.strategy(int(n), w) - os_.strategy(int(n), w))[:, own]
            assert diff.max() <= 1e-9, (n, w, diff.max())


def test_pcfrplus_checkpoint_resume_bitwise():
    spec, r = I.river_config(6)
    t = P.Tree(**spec)
    cfg = P.SolverConfig(variant="pcfr+")
    a = P.Solver(t, r, cfg)
    a.iterate(7)
    blob = a.save_state()
    a.iterate(8)
    b = P.Solver(t, r, cfg)
    b.load_state(blob)
    b.iterate(8)
    assert a.save_state() == b.save_state()
    np.testing.assert_array_equal(a.root_cfv("current"), b.root_cfv("current"))


def test_alternating_flop_network_leaves_runs_and_resumes():
    """Alternating updates with the network stage (two leaf batches per
    iteration): a checkpoint resume is bitwise and t counts iterations."""
    spec, r = I.flop_config(2, support=200)
    t = P.Tree(**spec)
    cfg = P.SolverConfig(alternating=1)
    a = P.Solver(t, r, cfg)
    n_leaves, n_next = a.leaf_rows()
    net = P.LeafNet(P.LEAF_D_IN, 64, 2, P.LEAF_D_OUT, max_batch=n_leaves * n_next)
    rng = np.random.default_rng(3)
    net.set_params([((rng.standard_normal((o, i)) / np.sqrt(i)).astype(np.float32), np.zeros(o, np.float32))
                    for o, i in net.layer_shapes()])
    a.attach_leafnet(net)
    a.iterate(5)
    blob = a.save_state()
    a.iterate(4)
    b = P.Solver(t, r, cfg)
    b.attach_leafnet(net)
    b.load_state(blob)
    b.iterate(4)
    assert a.t == 9 and b.t == 9
    assert a.save_state() == b.save_state()


@pytest.mark.parametrize("variant", ["dcfr", "pcfr+"])
@pytest.mark.parametrize("seed,support,spr", [(5, 40, 1.5), (7, 60, 1.0)])
def test_alternating_turn_matches_oracle(variant, seed, support, spr):
    """Alternating updates on turn trees (chance nodes), per iterate.

    FP64 parity with the oracle after 1, 3, 10 and 40 iterations: 1e-9 pot
    on root values (last iterate and average strategies), exploitability
    and both best responses; every average and current strategy entry of
    the hands in the acting player's support at every decision node within
    1e-9 through 10 iterations and 1e-7 at 40.  The strategies' bound widens
    with T because regret matching near ties amplifies rounding: a change
    of one ulp in the oracle's own input ranges moves its strategies by
    1e-13 after 3 iterations and by up to 6e-10 after 40 (measured on these
    four cases), and the GPU's sums, taken in another order, differ from
    the oracle's by rounding in every operation (measured: 1e-11 after 3
    iterations, 4e-11 after 10, 1.5e-8 after 40; root values 2e-12 pot).

    Player 1's half-step meets the exact zeros of player 0's new strategy at
    once: many of player 1's hands face opponents that all tie with them at
    a showdown, or no opponent hand with reach, so their actions' values tie
    exactly.  The oracle's sums over histories give exact zeros there; the
    GPU's prefix differences must too (counts of nonzero-reach hands decide
    when a win or loss sum is empty), or regret matching follows the signs
    of rounding residues and the runs part."""
    spec, r = I.turn_config(seed, support=support, spr=spr)
    say(f"case: alternating {variant} turn {spec} support {support}")
    ot = O.Tree.holdem(**spec)
    os_ = O.Solver(ot, r, support_only=True, variant=variant, alternating=True)
    gt = P.Tree(**spec)
    gs = P.Solver(gt, r, P.SolverConfig(dtype="f64", variant=variant, alternating=1))
    pot = spec["pot"]
    mask = (r > 0) & ~I.blocked_mask(spec["board"])[None, :]
    e = gt.export()
    dec = [int(n) for n in np.flatnonzero(e["type"] == P.NODE_DECISION)]
    for T in (1, 3, 10, 40):
        os_.iterate(T - os_.t)
        gs.iterate(T - gs.t)
        for which in ("current", "avg"):
            d = np.abs(gs.root_cfv(which) - os_.root_cfv(which))[mask].max() / pot
            say(f"  T={T} root cfv ({which}) max |d| = {d:.3e} pot")
            assert d <= 1e-9
        eg, bg = gs.exploitability()
        eo, bo = os_.exploitability()
        say(f"  T={T} exploitability gpu {eg:.12f} oracle {eo:.12f}")
        assert abs(eg - eo) / pot <= 1e-9
        np.testing.assert_allclose(bg / pot, bo / pot, atol=1e-9)
        worst = 0.0
        for n in dec:
            own = mask[int(e["player"][n])]
            for w in ("avg", "current"):
                worst = max(worst, float(np.abs(gs.strategy(n, w) - os_.strategy(n, w))[:, own].max()))
        say(f"  T={T} strategies (average and current) max |d| = {worst:.3e}")
        assert worst <= (1e-9 if T <= 10 else 1e-7)
