"""Leaf-network training on solver-generated turn subgames (GPU).

A small network is trained by the library's bf16 forward/backward/Adam
kernels on samples the batched solver produces; the test checks that the
Huber loss falls and that held-out value error (mbb/hand, hands weighted by
their own reach) ends below that of the best constant predictor fitted on
the training set, i.e. the network learned something about the solved
values; and that the trained network gains over the method without it.
Full-scale numbers come from paper_2605_19928_amd/leafnet_study.py.
"""
import numpy as np
import pytest

from paper_2605_19928_amd import pcfr as P
from paper_2605_19928_amd import train as T

pytestmark = pytest.mark.gpu


def test_training_reduces_loss_and_beats_constant():
    import torch
    X, Y, M, specs = T.generate(seed=11, n=192, iters=120, batch=64, log=print)
    assert torch.isfinite(Y).all() and (M.sum(dim=1) > 0).all()
    Xh, Yh, Mh, sh = T.generate(seed=12, n=32, iters=120, batch=32)
    net = P.LeafNet(P.LEAF_D_IN, 256, 2, P.LEAF_D_OUT, max_batch=256)
    rng = np.random.default_rng(0)
    params = [((rng.standard_normal((o, i)) * np.sqrt(2.0 / i)).astype(np.float32), np.zeros(o, np.float32))
              for o, i in net.layer_shapes()]
    net.set_params(params)
    hist = T.train(net, X, Y, M, steps=300, batch=128, lr=2e-3, log=print, log_every=50)
    assert hist[-1][1] < 0.5 * hist[0][1]
    pred = net.forward(Xh).cpu().numpy()
    pots = [s["pot"] for s, _ in sh]
    err_net, _ = T.value_error_mbb(pred, Yh.cpu().numpy(), Mh.cpu().numpy(), Xh.cpu().numpy(), pots)
    m = M.cpu().numpy()
    const = (Y.cpu().numpy() * m).sum(axis=0) / np.maximum(m.sum(axis=0), 1)
    err_const, _ = T.value_error_mbb(np.broadcast_to(const, pred.shape), Yh.cpu().numpy(), Mh.cpu().numpy(),
                                     Xh.cpu().numpy(), pots)
    print(f"held-out value error: network {err_net:.1f} mbb/hand, constant predictor {err_const:.1f} mbb/hand")
    assert err_net < err_const


def test_trained_network_beats_plain_solver_at_equal_time():
    """The gain test: on held-out turn subgames the trained network's values
    must be closer to the solved targets than the plain solver's after the
    iterations it can run in the network's evaluation time (at least one),
    and the plain solver's error must fall as it iterates (so the targets are
    reachable and the comparison is not rigged)."""
    import torch
    X, Y, M, _ = T.generate(seed=21, n=768, iters=150, batch=256, log=print)
    Xh, Yh, Mh, sh = T.generate(seed=22, n=48, iters=150, batch=48)
    net = P.LeafNet(P.LEAF_D_IN, 384, 2, P.LEAF_D_OUT, max_batch=256)
    rng = np.random.default_rng(1)
    net.set_params([((rng.standard_normal((o, i)) * np.sqrt(2.0 / i)).astype(np.float32), np.zeros(o, np.float32))
                    for o, i in net.layer_shapes()])
    T.train(net, X, Y, M, steps=800, batch=256, lr=2e-3, log=print, log_every=200)
    pots = [s["pot"] for s, _ in sh]
    pred = net.forward(Xh).cpu().numpy()
    e_net, _ = T.value_error_mbb(pred, Yh.cpu().numpy(), Mh.cpu().numpy(), Xh.cpu().numpy(), pots)
    t_net = T.forward_ms(net, Xh)
    curve, ms_iter = T.plain_solver_curve(sh, Yh, Mh, Xh, [1, 2, 4, 8, 16, 32, 64])
    k_eq = max(1, int(t_net // ms_iter))
    e_eq = [e for k, e in curve if k <= k_eq][-1]     # the plain solver's error within the network's time
    match = next((k for k, e in curve if e <= e_net), None)
    print(f"network: {e_net:.1f} mbb/hand in {t_net:.4f} ms; plain solver {ms_iter:.4f} ms/iteration, "
          f"errors {curve}; iterations in the network's time {t_net / ms_iter:.2f}; "
          f"iterations to match the network {match}")
    assert curve[-1][1] < curve[0][1]
    assert e_net < e_eq
