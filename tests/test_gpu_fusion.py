"""Terminal fusion: fold and showdown children evaluated inside their
parent's backward workgroup must give bitwise the iterates of the separate
terminal launch (same arithmetic, values read from LDS instead of memory),
on rivers, turns, batches, depth-limited trees with exact leaves, with every
Stage-7 rule, alternating updates, thresholding and pruning.  Compared as
arrays (a zero's sign is not part of an iterate)."""
import numpy as np
import pytest

from paper_2605_19928_amd import inputs as I
from paper_2605_19928_amd import pcfr as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def state(s, dtype):
    b = s.save_state()
    return np.frombuffer(b[16:], dtype=np.float64 if dtype == "f64" else np.float32)


def pair(make, T):
    a = make()            # fusion off (the default)
    b = make()
    b.set_terminal_fusion(True)
    a.iterate(T)
    b.iterate(T)
    return a, b


@pytest.mark.parametrize("case,dtype,variant,alt", [
    ("river", "f32", "dcfr", 0), ("river", "f64", "pcfr+", 1), ("turn", "f32", "dcfr", 0),
    ("turn", "f64", "cfr+", 0), ("turn", "f32", "pcfr+", 1), ("flop", "f32", "dcfr", 0), ("flop", "f64", "dcfr", 1)])
def test_fused_terminals_are_bitwise_the_separate_launch(case, dtype, variant, alt):
    if case == "river":
        spec, r = I.river_config(0)
    elif case == "turn":
        spec, r = I.turn_config(0, spr=2)
    else:
        spec, r = I.flop_config(0)
    say(f"case: terminal fusion, {case} {dtype} {variant} alternating={alt}")
    t = P.Tree(**spec)
    cfg = P.SolverConfig(dtype=dtype, variant=variant, alternating=alt)
    a, b = pair(lambda: P.Solver(t, r, cfg), 15)
    np.testing.assert_array_equal(state(a, dtype), state(b, dtype))
    np.testing.assert_array_equal(a.root_cfv("current"), b.root_cfv("current"))
    ea, _ = a.exploitability()
    eb, _ = b.exploitability()
    assert ea == eb


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fused_terminals_batch_threshold_prune(dtype):
    cases = I.batch_config(9, lambda sp: P.Tree(**sp).n_nodes, n=10, river_share=0.6, lo=10, hi=2000)
    trees = [P.Tree(**sp) for sp, _ in cases]
    ranges = np.stack([r for _, r in cases])
    say(f"case: terminal fusion, 10-subgame batch, threshold and pruning, {dtype}")
    cfg = P.SolverConfig(dtype=dtype, threshold=0.05, prune=1)
    a, b = pair(lambda: P.Batch(trees, ranges, cfg), 25)
    np.testing.assert_array_equal(state(a, dtype), state(b, dtype))
    for k in range(len(trees)):
        np.testing.assert_array_equal(a.root_cfv_of(k, "current"), b.root_cfv_of(k, "current"))


def test_fused_terminals_after_autotune():
    """The fusion plan follows the level-fusion schedule the autotuner picks."""
    spec, r = I.turn_config(0, spr=2)
    t = P.Tree(**spec)
    a = P.Solver(t, r)
    b = P.Solver(t, r)
    b.set_terminal_fusion(True)
    b.autotune(2)
    a.iterate(10)
    b.iterate(10)
    np.testing.assert_array_equal(state(a, "f32"), state(b, "f32"))
