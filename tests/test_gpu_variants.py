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
def test_alternating_turn_close_to_oracle(variant):
    """Alternating updates on a turn tree (chance nodes): per-iterate FP64
    parity does not hold here.  Below a chance node the library's regrets
    are K (= 44) times the oracle's -- it applies the chance probability
    1/K at the chance node, the oracle inside each history's weight -- which
    regret matching ignores; but after player 0's half-step some of player
    1's infosets carry regrets at rounding level, whose sign flips their
    strategy, and the two iterates drift apart (about 1e-3 pot after 40
    iterations on every seed tried).  What both reach is checked instead:
    the exploitability after 40 iterations within 5% of the oracle's
    (measured 0.1-2.2%), and below its value after one iteration."""
    spec, r = I.turn_config(5, support=40, spr=1.5)
    say(f"case: alternating {variant} turn {spec}")
    ot = O.Tree.holdem(**spec)
    os_ = O.Solver(ot, r, support_only=True, variant=variant, alternating=True)
    os_.iterate(40)
    gs = P.Solver(P.Tree(**spec), r, P.SolverConfig(dtype="f64", variant=variant, alternating=1))
    gs.iterate(1)
    e1, _ = gs.exploitability()
    gs.iterate(39)
    eg, _ = gs.exploitability()
    eo, _ = os_.exploitability()
    say(f"  exploitability after 40: gpu {eg:.6f} oracle {eo:.6f} (after 1: {e1:.4f}) chips/hand")
    assert abs(eg - eo) <= 0.05 * eo
    assert eg < e1
