"""Leaf-network training on subgames the solver itself solves.

The paper trains its leaf network as prior depth-limited solvers do (Sec. 2)
and values every depth-limit leaf with it (Sec. 3, Sec. 4.3 Stage 5).  Here:

1. ``generate``: random turn subgames (``inputs.leaf_training_config``) are
   solved in batches by the GPU solver; ``pcfr_batch_leaf_samples`` turns
   each solved subgame into one sample on the device (normalised ranges,
   board, stack-to-pot ratio -> each hand's value under the average
   strategies per pot and per unit of compatible opponent reach).
2. ``train``: Adam steps of the library's bf16-MFMA network on the Huber loss;
   each minibatch is relabelled by one random suit permutation (the game is
   suit-symmetric, so this is exact augmentation).
3. ``value_error_mbb``: error of predicted values in milli-big-blinds per hand
   (bb = 10 chips), weighting each hand by its own reach.

Only data movement (minibatch gathers, column permutations) uses torch; all
arithmetic of solving, sample building and training runs in the library.
"""
from __future__ import annotations

import itertools
import math
import time

import numpy as np

from . import inputs as I
from . import pcfr as P

NC = 1326
CC = I.combo_cards()


def suit_permutations():
    """Column index maps (input, output) for all 24 suit relabellings."""
    ins, outs = [], []
    for perm in itertools.permutations(range(4)):
        cmap = np.array([4 * (c // 4) + perm[c % 4] for c in range(52)])
        a, b = cmap[CC[:, 0]], cmap[CC[:, 1]]
        hi, lo = np.maximum(a, b), np.minimum(a, b)
        cidx = hi * (hi - 1) // 2 + lo                  # combo k -> relabelled combo
        src = np.empty(NC, dtype=np.int64)
        src[cidx] = np.arange(NC)                       # new column j reads old column src[j]
        card_src = np.empty(52, dtype=np.int64)
        card_src[cmap] = np.arange(52)
        xin = np.concatenate([src, NC + src, 2 * NC + card_src, [2 * NC + 52]])
        yout = np.concatenate([src, NC + src])
        ins.append(xin)
        outs.append(yout)
    return ins, outs


def generate(seed: int, n: int, iters: int, batch: int = 64, dtype: str = "f32", device="cuda", log=None,
             start: int = 0, **config):
    """Solve n random turn subgames (``inputs.leaf_training_config(seed, i, **config)``);
    return device tensors X [n, 2705], Y and M [n, 2652] and the cases."""
    import torch

    X = torch.zeros((n, P.LEAF_D_IN), dtype=torch.float32, device=device)
    Y = torch.zeros((n, P.LEAF_D_OUT), dtype=torch.float32, device=device)
    M = torch.zeros((n, P.LEAF_D_OUT), dtype=torch.float32, device=device)
    specs = []
    t0 = time.perf_counter()
    for b0 in range(0, n, batch):
        cases = [I.leaf_training_config(seed, start + i, **config) for i in range(b0, min(n, b0 + batch))]
        trees = [P.Tree(**s) for s, _ in cases]
        solver = P.Batch(trees, np.stack([r for _, r in cases]), P.SolverConfig(dtype=dtype), device=device)
        solver.iterate(iters)
        k = len(cases)
        solver.leaf_samples(X[b0:b0 + k], Y[b0:b0 + k], M[b0:b0 + k])
        specs.extend(cases)
        solver.close()
        if log:
            log(f"generate: {b0 + k}/{n} subgames solved ({time.perf_counter() - t0:.1f} s)")
    return X, Y, M, specs


def train(net: "P.LeafNet", X, Y, M, steps: int, batch: int = 1024, lr: float = 1e-3, seed: int = 0,
          augment: bool = True, log=None, log_every: int = 100):
    """Adam on the Huber loss with cosine learning-rate decay; returns the loss history."""
    import torch

    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    n = X.shape[0]
    ins, outs = suit_permutations()
    ins = [torch.as_tensor(a, device=X.device) for a in ins]
    outs = [torch.as_tensor(a, device=X.device) for a in outs]
    rng = np.random.default_rng(seed)
    hist = []
    for step in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), device=X.device, generator=g)
        xb, yb, mb = X[idx], Y[idx], M[idx]
        if augment:
            p = int(rng.integers(0, 24))
            xb, yb, mb = xb[:, ins[p]], yb[:, outs[p]], mb[:, outs[p]]
        cur = lr * 0.5 * (1 + math.cos(math.pi * step / max(steps, 1)))
        want = (step % log_every == 0) or step == steps - 1
        loss = net.train_step(xb, yb, mb, cur, want_loss=want)
        if want:
            hist.append((step, loss))
            if log:
                log(f"train: step {step} loss {loss:.6f} lr {cur:.2e}")
    return hist


def value_error_mbb(pred, Y, M, X, pots):
    """Mean over subgames of sum_i sum_h r_i(h) |pred - target| * pot * M_{-i}(h) / (2 Z), in mbb/hand.

    X carries each subgame's normalised ranges; M here is recomputed from them."""
    pred = np.asarray(pred, np.float64)
    Y = np.asarray(Y, np.float64)
    mk = np.asarray(M, np.float64)
    X = np.asarray(X, np.float64)
    out = []
    for g in range(X.shape[0]):
        r = X[g, :2 * NC].reshape(2, NC)
        card = np.zeros((2, 52))
        for p in range(2):
            np.add.at(card[p], CC[:, 0], r[p])
            np.add.at(card[p], CC[:, 1], r[p])
        mass = r.sum(axis=1)
        comp = [mass[o] - card[o][CC[:, 0]] - card[o][CC[:, 1]] + r[o] for o in range(2)]
        z = float((r[0] * comp[1]).sum())
        err = 0.0
        for i in range(2):
            d = np.abs(pred[g, i * NC:(i + 1) * NC] - Y[g, i * NC:(i + 1) * NC]) * mk[g, i * NC:(i + 1) * NC]
            err += float((r[i] * d * pots[g] * comp[1 - i]).sum())
        out.append(err / (2 * z) * 100.0)
    return float(np.mean(out)), out


def _elapsed_ms(fn, stream):
    import torch

    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def forward_ms(net: "P.LeafNet", X, reps: int = 20):
    """Device time of one network evaluation of the rows of X (ms)."""
    import torch

    net.forward(X)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(X.device)
    return _elapsed_ms(lambda: [net.forward(X) for _ in range(reps)], stream) / reps


def plain_solver_curve(cases, Yh, Mh, Xh, ks, dtype: str = "f32", device="cuda"):
    """The method without the network: the same held-out subgames solved by
    the plain batched solver for k iterations, for each k of the ascending
    ks; returns [(k, value error in mbb/hand of the average-strategy values
    against the targets)] and the device ms per batched iteration."""
    import torch

    trees = [P.Tree(**s) for s, _ in cases]
    b = P.Batch(trees, np.stack([r for _, r in cases]), P.SolverConfig(dtype=dtype), device=device)
    X = torch.zeros_like(Xh)
    Y = torch.zeros_like(Yh)
    Mk = torch.zeros_like(Mh)
    pots = [s["pot"] for s, _ in cases]
    yh, mh, xh = Yh.cpu().numpy(), Mh.cpu().numpy(), Xh.cpu().numpy()
    out, done, total = [], 0, 0.0
    for k in ks:
        total += _elapsed_ms(lambda: b.iterate(k - done), b.stream)
        done = k
        b.leaf_samples(X, Y, Mk)
        err, _ = value_error_mbb(Y.cpu().numpy(), yh, mh, xh, pots)
        out.append((int(k), float(err)))
    b.close()
    return out, total / max(done, 1)
