"""The benchmark's depth-limited flop with its full leaf network, end to end
against the oracle.

Workload: the flop of the benchmark (seed 0: pot 100, stacks 400, bet sizes
{33, 75}% + all-in, at most 3 per street), full Dirichlet(1) ranges, 21
network leaves x 49 next cards = 1029 network rows per iteration, the
2705 -> 4 x 1536 -> 2652 ReLU network with He-initialised weights (seeded),
bf16 operands and FP32 accumulation on the GPU.  The oracle builds every
leaf's network inputs from its own reach, runs the FP64 network with the
same bf16 operand roundings (oracle/mlp.py), applies the zero-sum shift,
and values the leaves history by history (Sec. 3, the depth-limited game).

Two checks, each for an FP32 and an FP64 tree:
* Steps from the oracle's trajectory: the oracle's state (t, regrets and
  average-strategy sums) after k = 0 .. 4 iterations is loaded into the GPU
  solver, both run one iteration, and the last-iterate root values, the
  reach-gated average strategies and the root values under the average
  strategies are held to 1e-4 pot; the exploitability of the resulting
  average strategy in the depth-limited game (leaves valued by the network
  on the average-strategy reach, on both sides) too.  This covers every
  kernel of the iteration at the benchmark's shapes on five states.
* Five free iterations from zero on both sides: the exploitability of the
  average strategy within 1e-4 pot.  Root values and strategies are printed,
  not asserted: hidden activations whose FP32 and FP64 sums straddle a bf16
  rounding boundary move single leaf values by a bf16 ulp, the next
  iteration's reach moves more inputs across rounding boundaries, and the
  early iterates of CFR amplify such differences (measured after five
  iterations: about 1.4e-4 pot on root values and 2e-2 on single gated
  strategy entries, in an FP64 tree as in an FP32 one, while the
  exploitability agrees to 1e-7 pot).
"""
import numpy as np
import pytest

import oracle as O
from oracle import mlp
from paper_2605_19928_amd import inputs as I
from paper_2605_19928_amd import pcfr as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def he_params(shapes, seed):
    rng = np.random.default_rng(seed)
    return [((rng.standard_normal((o, i)) * np.sqrt(2.0 / i)).astype(np.float32), np.zeros(o, np.float32))
            for o, i in shapes]


class Case:
    def __init__(self):
        self.spec, self.r = I.flop_config(0)
        self.ot = O.Tree.holdem(**self.spec)
        self.e = self.ot.export()
        self.leaves = np.flatnonzero(self.e["type"] == O.T_LEAF)
        self.ok = np.flatnonzero(~I.blocked_mask(self.spec["board"]))
        shapes = [(o, i) for o, i in mlp.layer_shapes(P.LEAF_D_IN, 1536, 4, P.LEAF_D_OUT)]
        self.params = he_params(shapes, 7)
        self.rs = np.concatenate([[0], np.cumsum(np.where(self.e["type"] == O.T_DEC, self.e["n_child"], 0))])

    def leaf_table(self, reach):
        """EV table [leaf][player][card][1326] of the network on the given per-node reach."""
        spec, e = self.spec, self.e
        eff = spec["stacks"][0]
        xs, cs = [], []
        for n in self.leaves:
            c = e["contrib"][n][0]
            cards, X = mlp.leaf_inputs(reach[n], spec["board"], pot=2 * c, stack_behind=spec["pot"] // 2 + eff - c,
                                       d_in=P.LEAF_D_IN)
            xs.append(X)
            cs.append(cards)
        Y = mlp.forward(self.params, np.concatenate(xs), emulate_bf16=True)
        ev = np.zeros((len(self.leaves), 2, 52, 1326))
        k0 = 0
        for li, n in enumerate(self.leaves):
            cards = cs[li]
            rows = np.stack([Y[k0:k0 + len(cards), :1326], Y[k0:k0 + len(cards), 1326:]], axis=1)
            rows = rows - mlp.zero_sum_shifts(rows, reach[n], cards)[:, None, None]
            ev[li][:, cards] = rows.transpose(1, 0, 2)
            k0 += len(cards)
        return ev

    def avg_reach(self, os_):
        """Reach of both players at every leaf under the oracle's average strategies."""
        e = self.e
        out = np.zeros((self.ot.n_nodes, 2, 1326))
        strat = {}
        for n in self.leaves:
            rr = self.r.copy()
            c = n
            while e["parent"][c] >= 0:
                p = int(e["parent"][c])
                if p not in strat:
                    strat[p] = os_.strategy(p, "avg")
                rr[int(e["player"][p])] *= strat[p][int(e["action"][c])]
                c = p
            out[n] = rr
        return out

    def step_oracle(self, os_):
        os_.set_leaf_table(self.leaf_table(os_.reach_current()))
        os_.iterate(1)

    def gpu(self, dtype):
        gt = P.Tree(**self.spec)
        gs = P.Solver(gt, self.r, P.SolverConfig(dtype=dtype))
        n_leaves, n_next = gs.leaf_rows()
        assert (n_leaves, n_next) == (21, 49)
        net = P.LeafNet(P.LEAF_D_IN, 1536, 4, P.LEAF_D_OUT, max_batch=n_leaves * n_next)
        net.set_params(self.params)
        gs.attach_leafnet(net)
        assert gt.n_hands == len(self.ok)
        return gt, gs, net

    def state_blob(self, os_, Hp, dtype):
        t = os_.t
        f = np.float32 if dtype == "f32" else np.float64
        parts = [np.array([t, np.dtype(f).itemsize], dtype=np.int64).tobytes()]
        for which in ("R", "S"):
            x = os_.rows(which)[:, self.ok]
            y = np.zeros((x.shape[0], Hp), dtype=f)
            y[:, :x.shape[1]] = x
            parts.append(y.tobytes())
        return b"".join(parts)

    def compare(self, gs, os_, tol, label, values=True, strategies=True):
        pot = self.spec["pot"]
        ok = self.ok
        dv = np.abs(gs.root_cfv("current") - os_.root_cfv("current"))[:, ok].max() / pot
        worst_g = 0.0
        S = os_.rows("S")
        for n in np.flatnonzero(self.e["type"] == O.T_DEC):
            d = np.abs(gs.strategy(int(n), "avg") - os_.strategy(int(n), "avg"))[:, ok]
            mass = S[self.rs[n]:self.rs[n] + self.e["n_child"][n]].sum(axis=0)[ok]
            gate = mass >= 1e-3 * max(mass.max(), 1e-300)
            if gate.any():
                worst_g = max(worst_g, float(d[:, gate].max()))
        # values and exploitability under the average strategies: the oracle's
        # leaves are valued by the network on the average-strategy reach, as the
        # GPU's evaluation sweeps value them
        os_.set_leaf_table(self.leaf_table(self.avg_reach(os_)))
        da = np.abs(gs.root_cfv("avg") - os_.root_cfv("avg"))[:, ok].max() / pot
        eg, bg = gs.exploitability()
        eo, bo = os_.exploitability()
        say(f"  {label}: root cfv (current) {dv:.3e}, (avg) {da:.3e} pot; gated avg strategy {worst_g:.3e}; "
            f"exploitability gpu {eg:.6f} oracle {eo:.6f} chips ({abs(eg - eo) / pot:.3e} pot)")
        if values:
            assert dv <= tol
            assert da <= tol
        if strategies:
            assert worst_g <= tol
        assert abs(eg - eo) / pot <= tol
        np.testing.assert_allclose(bg / pot, bo / pot, atol=tol)


@pytest.fixture(scope="module")
def case():
    return Case()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_bench_flop_steps_from_oracle_states(case, dtype):
    say(f"case: benchmark flop, full network, one step from the oracle's states k = 0..4, {dtype} tree")
    gt, gs, net = case.gpu(dtype)
    os_ = O.Solver(case.ot, case.r)
    for k in range(5):
        blob = case.state_blob(os_, gt.n_hands_padded, dtype)
        gs.load_state(blob)
        assert gs.t == k
        # the oracle's copy steps forward; its own trajectory continues from it
        ref = O.Solver(case.ot, case.r)
        ref.set_rows(os_.rows("R"), os_.rows("S"), k)
        case.step_oracle(ref)
        gs.iterate(1)
        case.compare(gs, ref, 1e-4, f"step {k} -> {k + 1}")
        case.step_oracle(os_)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_bench_flop_five_free_iterations(case, dtype):
    say(f"case: benchmark flop, full network, five free iterations, {dtype} tree")
    gt, gs, net = case.gpu(dtype)
    os_ = O.Solver(case.ot, case.r)
    for _ in range(5):
        case.step_oracle(os_)
    gs.iterate(5)
    case.compare(gs, os_, 1e-4, "after 5 iterations", values=False, strategies=False)
