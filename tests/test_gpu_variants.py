"""Stage-7 variants (CFR+, predictive CFR+) on the GPU vs the oracle.

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


@pytest.mark.parametrize("variant", ["cfr+", "pcfr+"])
@pytest.mark.parametrize("which", ["river", "turn"])
def test_variant_matches_oracle(variant, which):
    if which == "river":
        spec, r = I.river_config(4, support=140)
        so = False
    else:
        spec, r = I.turn_config(5, support=40, spr=1.5)
        so = True
    T = 40
    say(f"case: {variant} {which} {spec} T={T}")
    ot = O.Tree.holdem(**spec)
    os_ = O.Solver(ot, r, support_only=so, variant=variant)
    os_.iterate(T)
    gt = P.Tree(**spec)
    gs = P.Solver(gt, r, P.SolverConfig(dtype="f64", variant=variant))
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
