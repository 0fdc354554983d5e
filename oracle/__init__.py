"""FP64 CPU oracle for discounted CFR on hold'em public subgames.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never loads it, and it imports nothing from the product package.

The arithmetic lives in ``oracle.c`` (plain per-history CFR, written from the
paper's definitions in Sec. 3 and the seven-stage description of Sec. 4);
this module only loads the shared object and marshals arguments.

Parity status of each function (what pins it) is recorded in the tests under
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
NCOMBO = 1326

T_DEC, T_FOLD, T_SHOW, T_CHANCE, T_LEAF, T_ALLIN = range(6)


def build() -> str:
    """Compile the oracle with gcc (OpenMP, -O2)."""
    src = os.path.join(_HERE, "oracle.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
        sig = {
            "ora_eval5": (I, [P]),
            "ora_eval7": (I, [P]),
            "ora_category_counts": (None, [I, P]),
            "ora_distinct5": (I, []),
            "ora_eval7_batch": (None, [P, I64, P]),
            "ora_build_tree": (P, [I, P, I64, I64, I64, I, P, I, I, I]),
            "ora_build_kuhn": (P, []),
            "ora_tree_free": (None, [P]),
            "ora_tree_prune": (P, [P, P]),
            "ora_prune_dominated": (None, [P, P, P, P, P]),
            "ora_tree_info": (None, [P, P]),
            "ora_tree_export": (None, [P] * 10),
            "ora_solver_create": (P, [P, P, D, D, D, I]),
            "ora_solver_free": (None, [P]),
            "ora_iterate": (None, [P, I, I]),
            "ora_iteration": (I64, [P]),
            "ora_get_strategy": (I, [P, I, I, P]),
            "ora_get_rows": (None, [P, I, P]),
            "ora_set_rows": (None, [P, P, P, I64]),
            "ora_root_cfv_current": (None, [P, P]),
            "ora_root_cfv_avg": (None, [P, P]),
            "ora_pair_mass": (D, [P]),
            "ora_exploitability": (D, [P, P]),
            "ora_set_leaf_table": (None, [P, P]),
            "ora_num_leaves": (I, [P]),
            "ora_reach_current": (None, [P, P]),
            "ora_equity_table": (I, [P, I, P]),
            "ora_node_board": (I, [P, I, P]),
            "ora_set_traverser_hands": (None, [P, P]),
            "ora_max_threads": (I, []),
            "ora_set_variant": (None, [P, I]),
            "ora_set_alternating": (None, [P, I]),
            "ora_set_threshold": (None, [P, D]),
            "ora_canonical_flops": (I, [P, P, I]),
            "ora_set_flop_leaf_table": (I, [P, P]),
            "ora_has_flop_leaves": (I, [P]),
            "ora_leaf_cfv": (I, [P, I, I, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


N_CANONICAL_FLOPS = 1755


def canonical_flops():
    """The flops that no suit permutation maps to a smaller 52-bit card mask,
    by their sorted cards in lexicographic order, with the size of each one's
    orbit: (cards [1755, 3], orbit [1755])."""
    cards = np.zeros((N_CANONICAL_FLOPS, 3), dtype=np.int32)
    orbit = np.zeros(N_CANONICAL_FLOPS, dtype=np.int32)
    n = lib().ora_canonical_flops(_p(cards), _p(orbit), N_CANONICAL_FLOPS)
    assert n == N_CANONICAL_FLOPS
    return cards, orbit


def eval5(cards) -> int:
    a = np.ascontiguousarray(cards, dtype=np.int32)
    return int(lib().ora_eval5(_p(a)))


def eval7(cards) -> int:
    a = np.ascontiguousarray(cards, dtype=np.int32)
    return int(lib().ora_eval7(_p(a)))


def eval7_batch(cards: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(cards, dtype=np.int32).reshape(-1, 7)
    out = np.empty(a.shape[0], dtype=np.int32)
    lib().ora_eval7_batch(_p(a), a.shape[0], _p(out))
    return out


def category_counts(n: int) -> np.ndarray:
    out = np.zeros(9, dtype=np.int64)
    lib().ora_category_counts(n, _p(out))
    return out


def max_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().ora_max_threads())


def distinct5() -> int:
    return int(lib().ora_distinct5())


class Tree:
    """A public tree built by the oracle's own builder (breadth-first ids)."""

    def __init__(self, handle, kuhn=False):
        self._h = handle
        self.kuhn = kuhn
        info = np.zeros(9, dtype=np.int64)
        lib().ora_tree_info(self._h, _p(info))
        (self.n_nodes, self.n_decision, self.n_fold, self.n_showdown, self.n_chance,
         self.n_leaf, self.n_allin, self.n_levels, self.n_rows) = (int(x) for x in info)
        self.nh = 3 if kuhn else NCOMBO
        self.flop_leaves = bool(lib().ora_has_flop_leaves(self._h))

    @classmethod
    def holdem(cls, board, pot, stacks, sizes, allin=True, max_raises=2, depth_limit=0):
        b = np.asarray(board, dtype=np.int32)
        s = np.asarray(sizes, dtype=np.int32)
        h = lib().ora_build_tree(len(b), _p(b), int(pot), int(stacks[0]), int(stacks[1]),
                                 len(s), _p(s), int(allin), int(max_raises), int(depth_limit))
        if not h:
            raise ValueError("oracle rejected the tree spec")
        t = cls(h)
        t._keep = (b, s)
        return t

    @classmethod
    def kuhn_poker(cls):
        return cls(lib().ora_build_kuhn(), kuhn=True)

    def export(self) -> dict:
        n = self.n_nodes
        out = {k: np.zeros(n, dtype=np.int32) for k in
               ("type", "player", "parent", "action", "depth", "chance_card", "first_child", "n_child")}
        out["contrib"] = np.zeros((n, 2), dtype=np.int64)
        lib().ora_tree_export(self._h, _p(out["type"]), _p(out["player"]), _p(out["parent"]),
                              _p(out["action"]), _p(out["depth"]), _p(out["contrib"]),
                              _p(out["chance_card"]), _p(out["first_child"]), _p(out["n_child"]))
        return out

    def prune(self, removed):
        """The reduced game of online pruning (Sec. 5): removed[n] != 0 on a
        child of a decision node drops that action and its subtree.  Returns
        the reduced tree and, per node of this tree, its id in the reduced
        one (-1 when dropped)."""
        rm = np.ascontiguousarray(np.asarray(removed).astype(np.uint8))
        if rm.shape != (self.n_nodes,):
            raise ValueError("one flag per node")
        h = lib().ora_tree_prune(self._h, _p(rm))
        if not h:
            raise ValueError("invalid pruning flags")
        t = Tree(h, kuhn=self.kuhn)
        parent = self.export()["parent"]
        kept = np.zeros(self.n_nodes, dtype=bool)
        for n in range(self.n_nodes):
            kept[n] = not rm[n] and (parent[n] < 0 or kept[parent[n]])
        new_id = np.where(kept, np.cumsum(kept) - 1, -1).astype(np.int64)
        return t, new_id

    def prune_dominated(self, ranges, lo, hi) -> np.ndarray:
        """Flags of the actions online pruning removes (Sec. 5) given value
        bounds lo, hi [n_nodes][nh] indexed by the child node an action leads
        to: an action goes when, for every hand of the actor's range not
        blocked by the node's board, its upper bound lies below a sibling's
        lower bound."""
        r = np.ascontiguousarray(ranges, dtype=np.float64)
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        if r.shape != (2, self.nh) or lo.shape != (self.n_nodes, self.nh) or hi.shape != lo.shape:
            raise ValueError("ranges [2][nh], bounds [n_nodes][nh]")
        out = np.zeros(self.n_nodes, dtype=np.uint8)
        lib().ora_prune_dominated(self._h, _p(r), _p(lo), _p(hi), _p(out))
        return out

    def node_board(self, node: int) -> list:
        b = np.zeros(5, dtype=np.int32)
        nb = lib().ora_node_board(self._h, int(node), _p(b))
        return [int(x) for x in b[:nb]]

    def equity_table(self, node: int) -> np.ndarray:
        out = np.zeros((self.nh, self.nh), dtype=np.float64)
        if lib().ora_equity_table(self._h, int(node), _p(out)) != 0:
            raise ValueError("node has no board table")
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            lib().ora_tree_free(self._h)
            self._h = None


class Solver:
    """Per-history DCFR in FP64; simultaneous updates, or alternating ones
    (player 0, then player 1 against player 0's new strategy)."""

    VARIANTS = {"dcfr": 0, "cfr+": 1, "pcfr+": 2}

    def __init__(self, tree: Tree, ranges, alpha=1.5, beta=0.0, gamma=2.0, support_only=False, variant="dcfr",
                 alternating=False, threshold=0.0):
        self.tree = tree
        r = np.ascontiguousarray(ranges, dtype=np.float64).reshape(2, tree.nh)
        self._r = r
        self._h = lib().ora_solver_create(tree._h, _p(r), alpha, beta, gamma, int(support_only))
        lib().ora_set_variant(self._h, self.VARIANTS[variant])
        lib().ora_set_alternating(self._h, 1 if alternating else 0)
        if not (0.0 <= threshold < 1.0 / 12):
            raise ValueError("threshold must lie in [0, 1/12)")
        lib().ora_set_threshold(self._h, float(threshold))

    def _leaves_ready(self):
        if self.tree.flop_leaves and not getattr(self, "_flop_ev_set", False):
            raise ValueError("a preflop tree's leaves need a flop leaf table (set_flop_leaf_table)")

    def iterate(self, n: int, threads: int = 0):
        self._leaves_ready()
        lib().ora_iterate(self._h, int(n), int(threads))

    @property
    def t(self) -> int:
        return int(lib().ora_iteration(self._h))

    def strategy(self, node: int, which: str = "avg") -> np.ndarray:
        A = int(self.tree.export()["n_child"][node]) if not hasattr(self, "_nchild") else int(self._nchild[node])
        out = np.zeros((A, self.tree.nh), dtype=np.float64)
        if lib().ora_get_strategy(self._h, int(node), 0 if which == "avg" else 1, _p(out)) != 0:
            raise ValueError("not a decision node")
        return out

    def cache_shape(self):
        self._nchild = self.tree.export()["n_child"]
        return self

    def rows(self, which: str) -> np.ndarray:
        out = np.zeros((self.tree.n_rows, self.tree.nh), dtype=np.float64)
        lib().ora_get_rows(self._h, {"R": 0, "S": 1, "M": 2, "V": 3, "r": 4}[which], _p(out))
        return out

    def set_rows(self, R, S, t):
        R = np.ascontiguousarray(R, dtype=np.float64)
        S = np.ascontiguousarray(S, dtype=np.float64)
        lib().ora_set_rows(self._h, _p(R), _p(S), int(t))

    def root_cfv(self, which: str = "current") -> np.ndarray:
        self._leaves_ready()
        out = np.zeros((2, self.tree.nh), dtype=np.float64)
        if which == "current":
            lib().ora_root_cfv_current(self._h, _p(out))
        else:
            lib().ora_root_cfv_avg(self._h, _p(out))
        return out

    def pair_mass(self) -> float:
        return float(lib().ora_pair_mass(self._h))

    def exploitability(self):
        self._leaves_ready()
        br = np.zeros(2, dtype=np.float64)
        e = lib().ora_exploitability(self._h, _p(br))
        return float(e), br

    def num_leaves(self) -> int:
        return int(lib().ora_num_leaves(self._h))

    def set_flop_leaf_table(self, ev: np.ndarray):
        """Preflop trees: ev[leaf][player][flop][1326], expected values per
        unit of pot on the canonical flops (canonical_flops() order)."""
        ev = np.ascontiguousarray(ev, dtype=np.float64)
        assert ev.shape == (self.num_leaves(), 2, N_CANONICAL_FLOPS, self.tree.nh)
        if lib().ora_set_flop_leaf_table(self._h, _p(ev)) != 0:
            raise ValueError("the tree has no leaf at the flop deal")
        self._flop_ev_set = True

    def leaf_cfv(self, node: int, player: int, r_opp) -> np.ndarray:
        """Leaf node's counterfactual values of `player`'s hands against the
        opponent reach r_opp [1326] (sum over histories of reach x leaf value)."""
        self._leaves_ready()
        ro = np.ascontiguousarray(r_opp, dtype=np.float64)
        out = np.zeros(self.tree.nh, dtype=np.float64)
        if lib().ora_leaf_cfv(self._h, int(node), int(player), _p(ro), _p(out)) != 0:
            raise ValueError("not a leaf")
        return out

    def set_leaf_table(self, ev: np.ndarray):
        if self.tree.flop_leaves:
            raise ValueError("a preflop tree takes a flop leaf table")
        ev = np.ascontiguousarray(ev, dtype=np.float64)
        assert ev.size == self.num_leaves() * 2 * 52 * self.tree.nh
        self._ev = ev
        lib().ora_set_leaf_table(self._h, _p(ev))

    def set_traverser_hands(self, mask):
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(2, self.tree.nh)
        lib().ora_set_traverser_hands(self._h, _p(m))

    def reach_current(self) -> np.ndarray:
        out = np.zeros((self.tree.n_nodes, 2, self.tree.nh), dtype=np.float64)
        lib().ora_reach_current(self._h, _p(out))
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            lib().ora_solver_free(self._h)
            self._h = None
