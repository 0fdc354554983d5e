"""The allocation-free dominance test against the allocating one, through
the C ABI: identical flags (integer output, bit-exact) on two calls in a
row, the second on a smaller tree, so that the static scratch's leftovers
from the first call must not leak into the second; and a tree beyond the
scratch's limit is refused."""
import ctypes as C

import numpy as np
import pytest

from paper_2605_19928_amd import inputs as I
from paper_2605_19928_amd import pcfr as P

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def bounds(rng, e, spread=40.0, noise=10.0, width=5.0):
    n = len(e["type"])
    mid = rng.normal(size=(n, P.NCOMBO)) * noise
    for v in np.flatnonzero(e["type"] == P.NODE_DECISION):
        fc, A = int(e["first_child"][v]), int(e["n_child"][v])
        mid[fc: fc + A] += rng.normal(size=(A, 1)) * spread
    half = rng.random((n, P.NCOMBO)) * width
    return mid - half, mid + half


def test_noalloc_matches_allocating_entry_point_on_two_calls():
    rng = np.random.default_rng(21)
    cases = []
    board = [50, 46, 26, 10]
    spec = dict(board=board, pot=100, stacks=(300, 300), sizes=[50, 100], allin=True, max_raises=2, depth_limit=0)
    r = np.stack([I.dirichlet_range(rng, board, support=300), I.dirichlet_range(rng, board, support=300)])
    cases.append((spec, r))
    cases.append(I.river_config(2, support=200))          # second call: a smaller tree
    sizes = []
    for spec, r in cases:
        t = P.Tree(**spec)
        print(f"case: noalloc dominance, board={spec['board']} nodes={t.n_nodes}", flush=True)
        lo, hi = bounds(rng, t.export())
        dlo, dhi = _dev(lo), _dev(hi)
        want = t.prune_dominated(r, dlo, dhi)
        got = t.prune_dominated(r, dlo, dhi, noalloc=True)
        assert want.sum() > 0
        np.testing.assert_array_equal(got, want)
        sizes.append(t.n_nodes)
    assert sizes[1] < sizes[0]


def test_noalloc_refuses_trees_beyond_its_scratch():
    spec, r = I.turn_config(0)           # 77,529 nodes but 27,524 decision nodes: fits
    t = P.Tree(**spec)
    assert t.n_nodes <= 262144 and t.n_decision <= 65536
    big = P.Tree(board=spec["board"][:3], pot=100, stacks=(400, 400), sizes=[33, 75], allin=True, max_raises=3,
                 depth_limit=0)         # the flop dealt out to showdown: millions of nodes
    assert big.n_nodes > 262144
    # the size check runs on the host before anything is launched, so the
    # one-row bound tensors are never read
    z = _dev(np.zeros((1, P.NCOMBO)))
    out = np.zeros(big.n_nodes, dtype=np.uint8)
    rr = np.zeros((2, P.NCOMBO))
    rc = P.lib().pcfr_prune_dominated_noalloc(big._h, P._p(rr), C.c_void_p(z.data_ptr()), C.c_void_p(z.data_ptr()),
                                              P._p(out))
    assert rc == P.E_TOO_LARGE
