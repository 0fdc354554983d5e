"""Python binding of ``libpcfr.so`` (argument marshalling only).

Every step of a CFR iteration runs in the library's HIP kernels; this module
only converts arguments, owns the device workspace as a torch tensor, and
passes torch's current stream.  If the built library is missing, importing
the binding raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcfr.so")
NCOMBO = 1326

OK, E_INVALID_ARG, E_OUT_OF_MEMORY, E_DEVICE, E_STATE, E_UNSUPPORTED, E_NUMERIC, E_TOO_LARGE = range(8)
F32, F64 = 0, 1
AVG, CURRENT = 0, 1
DCFR, CFRPLUS, PCFRPLUS = 0, 1, 2
NODE_DECISION, NODE_FOLD, NODE_SHOWDOWN, NODE_CHANCE, NODE_LEAF, NODE_ALLIN_LEAF = range(6)


class PcfrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pcfr error {code}: {msg}")
        self.code = code


class TreeSpec(C.Structure):
    _fields_ = [("n_board", C.c_int32), ("board", C.c_int32 * 5), ("pot", C.c_int64),
                ("stack", C.c_int64 * 2), ("n_sizes", C.c_int32), ("size_pct", C.c_int32 * 8),
                ("allin", C.c_int32), ("max_raises", C.c_int32), ("depth_limit", C.c_int32)]


class SolverCfg(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("variant", C.c_int32), ("alpha", C.c_double),
                ("beta", C.c_double), ("gamma", C.c_double), ("alternating", C.c_int32), ("suit_iso", C.c_int32),
                ("threshold", C.c_double), ("prune", C.c_int32)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "pcfr_abi_version": (C.c_int32, []),
    "pcfr_last_error": (C.c_char_p, []),
    "pcfr_build_tree": (C.c_int32, [C.POINTER(TreeSpec), C.POINTER(C.c_void_p)]),
    "pcfr_tree_free": (C.c_int32, [C.c_void_p]),
    "pcfr_tree_info": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pcfr_tree_export": (C.c_int32, [C.c_void_p] * 10),
    "pcfr_eval7_batch": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p]),
    "pcfr_suit_iso_map": (C.c_int32, [C.c_void_p] * 6),
    "pcfr_prune_dominated": (C.c_int32, [C.c_void_p] * 5),
    "pcfr_prune_dominated_noalloc": (C.c_int32, [C.c_void_p] * 5),
    "pcfr_solver_set_launch": (C.c_int32, [C.c_void_p, C.c_int32]),
    "pcfr_solver_set_terminal_fusion": (C.c_int32, [C.c_void_p, C.c_int32]),
    "pcfr_solver_unreached_nodes": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)]),
    "pcfr_tree_prune": (C.c_int32, [C.c_void_p] * 4),
    "pcfr_solver_swept_nodes": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)]),
    "pcfr_equity_table": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pcfr_leafnet_workspace_bytes": (C.c_int32, [C.c_int32] * 5 + [C.POINTER(C.c_size_t)]),
    "pcfr_leafnet_create": (C.c_int32, [C.c_int32] * 5 + [C.c_void_p, C.c_size_t, C.c_void_p,
                                                          C.POINTER(C.c_void_p)]),
    "pcfr_leafnet_free": (C.c_int32, [C.c_void_p]),
    "pcfr_leafnet_num_params": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)]),
    "pcfr_leafnet_set_params": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pcfr_leafnet_get_params": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pcfr_leafnet_get_grads": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pcfr_leafnet_forward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "pcfr_leafnet_train_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                            C.c_float, C.POINTER(C.c_float)]),
    "pcfr_solver_attach_leafnet": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pcfr_solver_set_leaf_zero_sum": (C.c_int32, [C.c_void_p, C.c_int32]),
    "pcfr_batch_workspace_bytes": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(SolverCfg), C.POINTER(C.c_size_t)]),
    "pcfr_batch_create": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(SolverCfg), C.c_void_p, C.c_void_p,
                                      C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pcfr_batch_size": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32)]),
    "pcfr_batch_get_strategy": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "pcfr_batch_get_root_cfv": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "pcfr_batch_exploitability": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pcfr_batch_leaf_samples": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    "pcfr_leaf_rows": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "pcfr_solver_workspace_bytes": (C.c_int32, [C.c_void_p, C.POINTER(SolverCfg), C.POINTER(C.c_size_t)]),
    "pcfr_solver_create": (C.c_int32, [C.c_void_p, C.POINTER(SolverCfg), C.c_void_p, C.c_void_p, C.c_size_t,
                                       C.c_void_p, C.POINTER(C.c_void_p)]),
    "pcfr_solver_free": (C.c_int32, [C.c_void_p]),
    "pcfr_cfr_iterate": (C.c_int32, [C.c_void_p, C.c_int32]),
    "pcfr_synchronize": (C.c_int32, [C.c_void_p]),
    "pcfr_profile_iterations": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "pcfr_autotune": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pcfr_batch_autotune": (C.c_int32, [C.c_void_p, C.c_int32]),
    "pcfr_leafnet_autotune": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]),
    "pcfr_leafnet_set_tiles": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32]),
    "pcfr_leafnet_get_tiles": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32]),
    "pcfr_iteration": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)]),
    "pcfr_get_strategy": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "pcfr_get_root_cfv": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "pcfr_node_values": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "pcfr_exploitability": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "pcfr_state_bytes": (C.c_int32, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "pcfr_save_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "pcfr_load_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
}


def lib():
    """Load the built library; raises if it was not built.

    torch is imported first: its wheel carries its own HIP runtime under the
    same soname, and the device memory and streams this binding passes come
    from torch, so the library must bind to that runtime rather than load a
    second one."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads torch's HIP runtime before libpcfr.so)

        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_19928_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc: int):
    if rc != OK:
        raise PcfrError(rc, lib().pcfr_last_error().decode(errors="replace"))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def eval7_batch(cards) -> np.ndarray:
    a = np.ascontiguousarray(cards, dtype=np.int32).reshape(-1, 7)
    out = np.empty(a.shape[0], dtype=np.int32)
    _check(lib().pcfr_eval7_batch(_p(a), a.shape[0], _p(out)))
    return out


class Tree:
    """Public tree of a subgame, built on the host by the library."""

    def __init__(self, board, pot, stacks, sizes, allin=True, max_raises=2, depth_limit=0):
        sp = TreeSpec()
        sp.n_board = len(board)
        for i, c in enumerate(board):
            sp.board[i] = int(c)
        sp.pot = int(pot)
        sp.stack[0], sp.stack[1] = int(stacks[0]), int(stacks[1])
        if len(sizes) > 8:
            raise ValueError("at most 8 bet sizes")
        sp.n_sizes = len(sizes)
        for i, s in enumerate(sizes):
            sp.size_pct[i] = int(s)
        sp.allin, sp.max_raises, sp.depth_limit = int(allin), int(max_raises), int(depth_limit)
        h = C.c_void_p()
        _check(lib().pcfr_build_tree(C.byref(sp), C.byref(h)))
        self._h = h
        self.spec = dict(board=list(board), pot=pot, stacks=tuple(stacks), sizes=list(sizes), allin=allin,
                         max_raises=max_raises, depth_limit=depth_limit)
        self._load_info()

    def _load_info(self):
        info = np.zeros(16, dtype=np.int64)
        _check(lib().pcfr_tree_info(self._h, _p(info)))
        (self.n_nodes, self.n_decision, self.n_fold, self.n_showdown, self.n_chance, self.n_leaf,
         self.n_allin, self.n_levels, self.n_rows, self.n_hands, self.n_hands_padded) = (int(x) for x in info[:11])

    def equity_table(self) -> np.ndarray:
        out = np.zeros((NCOMBO, NCOMBO), dtype=np.float64)
        _check(lib().pcfr_equity_table(self._h, _p(out)))
        return out

    def suit_iso_map(self, ranges) -> dict:
        """The library's suit isomorphism map for root ranges [2, 1326]: group
        (bitmask over the 24 suit permutations), per node src, perm, skip."""
        r = np.ascontiguousarray(ranges, dtype=np.float64).reshape(2, NCOMBO)
        n = self.n_nodes
        grp = C.c_uint32()
        src = np.zeros(n, dtype=np.int32)
        perm = np.zeros(n, dtype=np.int32)
        skip = np.zeros(n, dtype=np.int8)
        _check(lib().pcfr_suit_iso_map(self._h, _p(r), C.byref(grp), _p(src), _p(perm), _p(skip)))
        return {"group": int(grp.value), "src": src, "perm": perm, "skip": skip}

    def prune_dominated(self, ranges, lo, hi, noalloc: bool = False) -> np.ndarray:
        """Dominance test of online pruning on the GPU.  lo, hi: CUDA float64
        tensors [n_nodes, 1326] of bounds on the actor's value of the action
        leading to each node.  Returns uint8 flags [n_nodes]: 1 where that
        action is dominated for every hand of the actor's range.  noalloc:
        use the entry point that allocates no device memory."""
        import torch

        r = np.ascontiguousarray(ranges, dtype=np.float64).reshape(2, NCOMBO)
        for b in (lo, hi):
            if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.float64
                    and b.is_contiguous() and tuple(b.shape) == (self.n_nodes, NCOMBO)):
                raise ValueError("bounds must be contiguous CUDA float64 tensors [n_nodes, 1326]")
        torch.cuda.current_stream(lo.device).synchronize()
        out = np.zeros(self.n_nodes, dtype=np.uint8)
        fn = lib().pcfr_prune_dominated_noalloc if noalloc else lib().pcfr_prune_dominated
        _check(fn(self._h, _p(r), C.c_void_p(lo.data_ptr()), C.c_void_p(hi.data_ptr()), _p(out)))
        return out

    def prune(self, removed):
        """The reduced tree without the flagged actions and their subtrees,
        and each node's id in it (-1 when dropped)."""
        rm = np.ascontiguousarray(np.asarray(removed).astype(np.uint8))
        if rm.shape != (self.n_nodes,):
            raise ValueError("one flag per node")
        new_id = np.zeros(self.n_nodes, dtype=np.int32)
        h = C.c_void_p()
        _check(lib().pcfr_tree_prune(self._h, _p(rm), C.byref(h), _p(new_id)))
        t = Tree.__new__(Tree)
        t._h = h
        t.spec = dict(self.spec)
        t._load_info()
        return t, new_id

    def export(self) -> dict:
        n = self.n_nodes
        out = {k: np.zeros(n, dtype=np.int32) for k in
               ("type", "player", "parent", "action", "depth", "chance_card", "first_child", "n_child")}
        out["contrib"] = np.zeros((n, 2), dtype=np.int64)
        _check(lib().pcfr_tree_export(self._h, _p(out["type"]), _p(out["player"]), _p(out["parent"]),
                                      _p(out["action"]), _p(out["depth"]), _p(out["contrib"]),
                                      _p(out["chance_card"]), _p(out["first_child"]), _p(out["n_child"])))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pcfr_tree_free(h)
            self._h = None


VARIANTS = {"dcfr": DCFR, "cfr+": CFRPLUS, "pcfr+": PCFRPLUS}


@dataclass
class SolverConfig:
    dtype: str = "f32"
    alpha: float = 1.5
    beta: float = 0.0
    gamma: float = 2.0
    variant: str = "dcfr"
    alternating: int = 0
    suit_iso: int = 0
    threshold: float = 0.0
    prune: int = 0

    def to_c(self) -> SolverCfg:
        c = SolverCfg()
        c.dtype = F64 if self.dtype == "f64" else F32
        v = VARIANTS[self.variant] if isinstance(self.variant, str) else int(self.variant)
        c.variant, c.alpha, c.beta, c.gamma, c.alternating, c.suit_iso = (v, self.alpha, self.beta, self.gamma,
                                                                         self.alternating, self.suit_iso)
        c.threshold, c.prune = float(self.threshold), int(self.prune)
        return c


class Solver:
    """DCFR solver on the GPU.  The workspace is a torch uint8 tensor on
    ``device``; work is enqueued on torch's current stream of that device."""

    def __init__(self, tree: Tree, ranges, cfg: SolverConfig | None = None, device="cuda"):
        import torch

        self.tree = tree
        self.cfg = cfg or SolverConfig()
        c = self.cfg.to_c()
        self._cfg_c = c
        nbytes = C.c_size_t()
        _check(lib().pcfr_solver_workspace_bytes(tree._h, C.byref(c), C.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self.device = torch.device(device)
        self.ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.ws.data_ptr()
        ptr = (ptr + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        r = np.ascontiguousarray(ranges, dtype=np.float64).reshape(2, NCOMBO)
        self._ranges = r
        h = C.c_void_p()
        _check(lib().pcfr_solver_create(tree._h, C.byref(c), _p(r), C.c_void_p(ptr),
                                        self.workspace_bytes, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self._nchild = tree.export()["n_child"]

    def iterate(self, n: int):
        _check(lib().pcfr_cfr_iterate(self._h, int(n)))

    def swept_nodes(self) -> int:
        """Nodes the sweeps visit (fewer than the tree's with suit isomorphism)."""
        n = C.c_int64()
        _check(lib().pcfr_solver_swept_nodes(self._h, C.byref(n)))
        return int(n.value)

    def profile(self, n: int):
        """Run n iterations with per-launch event timing; returns (ms[8], launches[8])
        for the classes bookkeeping, forward, terminal, backward, leaves, leaf GEMMs."""
        ms = np.zeros(8, dtype=np.float64)
        cnt = np.zeros(8, dtype=np.int64)
        _check(lib().pcfr_profile_iterations(self._h, int(n), _p(ms), _p(cnt)))
        return ms, cnt

    def autotune(self, reps: int = 5):
        """Pick each level sweep's workgroup size by timing (fresh solvers only);
        returns ms per iteration (before, after).  The state is left at t = 0."""
        a, b = C.c_double(), C.c_double()
        _check(lib().pcfr_autotune(self._h, int(reps), C.byref(a), C.byref(b)))
        return float(a.value), float(b.value)

    def autotune_budget(self, budget_ms: int = 200):
        """The autotuner within a device-time budget (fresh solvers only)."""
        _check(lib().pcfr_batch_autotune(self._h, int(budget_ms)))

    def set_launch(self, persistent: bool):
        """Run iterate(n) as one persistent cooperative launch (True) or as
        graph replays of per-level launches (False, the default); the iterates
        are bitwise the same."""
        _check(lib().pcfr_solver_set_launch(self._h, 1 if persistent else 0))

    def set_terminal_fusion(self, on: bool):
        """Evaluate fold/showdown children inside their parent's backward launch (default off)."""
        _check(lib().pcfr_solver_set_terminal_fusion(self._h, 1 if on else 0))

    def unreached_nodes(self) -> int:
        """Nodes the last iteration skipped as unreachable (solvers with prune=1)."""
        n = C.c_int64()
        _check(lib().pcfr_solver_unreached_nodes(self._h, C.byref(n)))
        return int(n.value)

    def synchronize(self):
        _check(lib().pcfr_synchronize(self._h))

    @property
    def t(self) -> int:
        v = C.c_int64()
        _check(lib().pcfr_iteration(self._h, C.byref(v)))
        return int(v.value)

    def strategy(self, node: int, which: str = "avg") -> np.ndarray:
        A = int(self._nchild[node])
        out = np.zeros((max(A, 1), NCOMBO), dtype=np.float64)
        _check(lib().pcfr_get_strategy(self._h, int(node), AVG if which == "avg" else CURRENT, _p(out)))
        return out

    def root_cfv(self, which: str = "current") -> np.ndarray:
        out = np.zeros((2, NCOMBO), dtype=np.float64)
        _check(lib().pcfr_get_root_cfv(self._h, CURRENT if which == "current" else AVG, _p(out)))
        return out

    def node_values(self, sub: int = 0):
        """Counterfactual values of every node under the average strategies:
        CUDA float64 tensor [n_nodes, 2, 1326]."""
        import torch

        n = self.tree.n_nodes if not hasattr(self, "trees") else self.trees[sub].n_nodes
        out = torch.zeros((n, 2, NCOMBO), dtype=torch.float64, device=self.device)
        self.stream.synchronize()
        _check(lib().pcfr_node_values(self._h, int(sub), C.c_void_p(out.data_ptr())))
        return out

    def exploitability(self):
        e = C.c_double()
        br = np.zeros(2, dtype=np.float64)
        _check(lib().pcfr_exploitability(self._h, C.byref(e), _p(br)))
        return float(e.value), br

    def save_state(self) -> bytes:
        n = C.c_size_t()
        _check(lib().pcfr_state_bytes(self._h, C.byref(n)))
        buf = (C.c_char * n.value)()
        _check(lib().pcfr_save_state(self._h, buf, n.value))
        return bytes(buf)

    def load_state(self, blob: bytes):
        buf = (C.c_char * len(blob)).from_buffer_copy(blob)
        _check(lib().pcfr_load_state(self._h, buf, len(blob)))

    def attach_leafnet(self, net: "LeafNet | None"):
        _check(lib().pcfr_solver_attach_leafnet(self._h, net._h if net is not None else None))
        self._net = net

    def set_leaf_zero_sum(self, on: bool):
        """Shift network leaf values to zero-sum per (leaf, next card) (default on)."""
        _check(lib().pcfr_solver_set_leaf_zero_sum(self._h, 1 if on else 0))

    def leaf_rows(self):
        a, b = C.c_int32(), C.c_int32()
        _check(lib().pcfr_leaf_rows(self._h, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pcfr_solver_free(h)
            self._h = None

    def __del__(self):
        self.close()


class Batch(Solver):
    """Many subgames advanced together by the same launches (one forest)."""

    def __init__(self, trees, ranges, cfg: SolverConfig | None = None, device="cuda"):
        import torch

        self.trees = list(trees)
        self.tree = self.trees[0]
        self.cfg = cfg or SolverConfig()
        c = self.cfg.to_c()
        self._cfg_c = c
        n = len(self.trees)
        arr = (C.c_void_p * n)(*[t._h.value for t in self.trees])
        self._arr = arr
        nbytes = C.c_size_t()
        _check(lib().pcfr_batch_workspace_bytes(arr, n, C.byref(c), C.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self.device = torch.device(device)
        self.ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        r = np.ascontiguousarray(ranges, dtype=np.float64).reshape(n, 2, NCOMBO)
        self._ranges = r
        h = C.c_void_p()
        _check(lib().pcfr_batch_create(arr, n, C.byref(c), _p(r), C.c_void_p(ptr), self.workspace_bytes,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self._nchildren = [t.export()["n_child"] for t in self.trees]
        self._nchild = self._nchildren[0]
        self.n = n

    def strategy_of(self, sub: int, node: int, which: str = "avg") -> np.ndarray:
        A = int(self._nchildren[sub][node])
        out = np.zeros((max(A, 1), NCOMBO), dtype=np.float64)
        _check(lib().pcfr_batch_get_strategy(self._h, int(sub), int(node), AVG if which == "avg" else CURRENT,
                                             _p(out)))
        return out

    def root_cfv_of(self, sub: int, which: str = "current") -> np.ndarray:
        out = np.zeros((2, NCOMBO), dtype=np.float64)
        _check(lib().pcfr_batch_get_root_cfv(self._h, int(sub), CURRENT if which == "current" else AVG, _p(out)))
        return out

    def leaf_samples(self, X, Y, Mk):
        """Fill rows of device tensors X [n, >=2705], Y and Mk [n, >=2652] (fp32) with one
        leaf-network sample per subgame (values under the average strategies)."""
        for t in (X, Y, Mk):
            assert t.is_contiguous() and t.shape[0] >= self.n
        _check(lib().pcfr_batch_leaf_samples(self._h, C.c_void_p(X.data_ptr()), int(X.shape[1]),
                                             C.c_void_p(Y.data_ptr()), C.c_void_p(Mk.data_ptr()), int(Y.shape[1])))

    def exploitability_all(self):
        e = np.zeros(self.n, dtype=np.float64)
        br = np.zeros((self.n, 2), dtype=np.float64)
        _check(lib().pcfr_batch_exploitability(self._h, _p(e), _p(br)))
        return e, br


LEAF_D_IN = 2 * NCOMBO + 53
LEAF_D_OUT = 2 * NCOMBO


class LeafNet:
    """ReLU MLP on the GPU (bf16 MFMA GEMMs, FP32 masters, Adam)."""

    def __init__(self, d_in=LEAF_D_IN, width=1536, depth=4, d_out=LEAF_D_OUT, max_batch=2048, device="cuda"):
        import torch

        self.shape = (d_in, width, depth, d_out)
        nbytes = C.c_size_t()
        _check(lib().pcfr_leafnet_workspace_bytes(d_in, width, depth, d_out, max_batch, C.byref(nbytes)))
        self.device = torch.device(device)
        self.ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().pcfr_leafnet_create(d_in, width, depth, d_out, max_batch, C.c_void_p(ptr), int(nbytes.value),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        n = C.c_int64()
        _check(lib().pcfr_leafnet_num_params(self._h, C.byref(n)))
        self.n_params = int(n.value)

    def layer_shapes(self):
        d_in, width, depth, d_out = self.shape
        dims = [d_in] + [width] * depth + [d_out]
        return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]

    def set_params(self, layers):
        """layers: list of (W [out, in], b [out]) arrays."""
        flat = np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()])
                               for W, b in layers]).astype(np.float32)
        assert flat.size == self.n_params
        _check(lib().pcfr_leafnet_set_params(self._h, _p(flat)))

    def _unflat(self, flat):
        out, k = [], 0
        for o, i in self.layer_shapes():
            W = flat[k:k + o * i].reshape(o, i)
            k += o * i
            b = flat[k:k + o]
            k += o
            out.append((W, b))
        return out

    def get_params(self):
        flat = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().pcfr_leafnet_get_params(self._h, _p(flat)))
        return self._unflat(flat)

    def get_grads(self):
        flat = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().pcfr_leafnet_get_grads(self._h, _p(flat)))
        return self._unflat(flat)

    def forward(self, x):
        """x: torch float32 [m, d_in] on the device -> torch float32 [m, d_out]."""
        import torch

        x = x.contiguous()
        y = torch.empty((x.shape[0], self.shape[3]), dtype=torch.float32, device=self.device)
        _check(lib().pcfr_leafnet_forward(self._h, C.c_void_p(x.data_ptr()), int(x.shape[0]),
                                          C.c_void_p(y.data_ptr())))
        return y

    def autotune(self, m: int, reps: int = 10):
        """Pick each forward layer's GEMM tile for m-row batches; returns ms per forward (before, after)."""
        a, b = C.c_double(), C.c_double()
        _check(lib().pcfr_leafnet_autotune(self._h, int(m), int(reps), C.byref(a), C.byref(b)))
        return float(a.value), float(b.value)

    @property
    def tiles(self):
        """Forward GEMM tile per layer (-1 default, 0 64x64, 1 128x64, 2 64x128, 3 128x128,
        4 64x64 and 5 64x128 with the K loop split between two wave groups, 6 64x64 and
        7 64x128 with a deeper prefetch, 8, 9 and 10 direct tiles reading operands straight
        into registers, 9 and 10 with K split in two and four; direct tiles only as a suffix
        of layers after the first)."""
        t = np.zeros(len(self.layer_shapes()), dtype=np.int32)
        _check(lib().pcfr_leafnet_get_tiles(self._h, _p(t), len(t)))
        return [int(v) for v in t]

    @tiles.setter
    def tiles(self, tiles):
        t = np.ascontiguousarray(tiles, dtype=np.int32)
        _check(lib().pcfr_leafnet_set_tiles(self._h, _p(t), len(t)))

    def train_step(self, x, target, mask, lr: float, want_loss: bool = True):
        loss = C.c_float()
        _check(lib().pcfr_leafnet_train_step(self._h, C.c_void_p(x.contiguous().data_ptr()),
                                             C.c_void_p(target.contiguous().data_ptr()),
                                             C.c_void_p(mask.contiguous().data_ptr()), int(x.shape[0]), float(lr),
                                             C.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pcfr_leafnet_free(h)
            self._h = None

    def __del__(self):
        self.close()
