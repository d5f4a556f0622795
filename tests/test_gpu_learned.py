"""Learned warm start on the GPU.

1. The pipeline end to end on a small sample: generate solves with the plain
   batched method, train the network with the project's kernels (the loss must
   fall), warm-start held-out problems through nrto_warm_start.
2. What the network trained on 20k solves (the committed weights) gains over
   the method without it on held-out problems: fewer DR iterations where both
   starts converge, with the cold fallback in place and nearly as many
   converged solves."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2603_02642_amd", "weights", "ws_quadrotor_T50.npz")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_learned_pipeline_small():
    torch = _torch()
    from paper_2603_02642_amd import learned as L
    from paper_2603_02642_amd import nrto
    opt = L.dr_options(max_admm=200)
    X, Y, ok = L.generate(192, chunk=192, opt=opt, log=lambda *a: None)
    assert ok.sum() >= 96
    losses = []
    net, norm = L.train(X[ok], Y[ok], epochs=30, batch=64, log=lambda m: losses.append(float(m.split()[-1])))
    assert losses[-1] < 0.8 * losses[0]
    probs = L.problems("heldout", 0, 16)
    ctx = nrto.Context(probs, opt)
    ctx.linearize()
    pred = net.infer(torch.from_numpy(L.features(probs)).cuda())
    acc, res = ctx.warm_start(pred, gains=False)
    assert acc.shape == (16,) and np.all(np.isfinite(res))
    # the fallback keeps the cold point exactly where the warm one is worse
    assert np.all((acc == 1) == (res[:, 0] <= res[:, 1]))
    warm = ctx.solve(warm=True)
    assert sum(r.kkt <= 1e-4 for r in warm) >= 8


def test_trained_network_gain_over_cold_start():
    torch = _torch()
    from paper_2603_02642_amd import learned as L
    from paper_2603_02642_amd import nrto
    opt = L.dr_options(max_admm=200)
    probs = L.problems("heldout", 0, 64)
    ctx = nrto.Context(probs, opt)
    ctx.linearize()
    cold = ctx.solve()
    net = L.load_net(WEIGHTS, max_batch=64)
    pred = net.infer(torch.from_numpy(L.features(probs)).cuda())
    acc, res = ctx.warm_start(pred, gains=L.rows_have_gains(WEIGHTS))
    warm = ctx.solve(warm=True)
    ok_c = np.array([r.kkt <= 1e-4 for r in cold])
    ok_w = np.array([r.kkt <= 1e-4 for r in warm])
    assert ok_w.sum() >= ok_c.sum() - 6
    both = ok_c & ok_w
    assert both.sum() >= 48
    it_cold = np.mean([r.inner_iters for r, b in zip(cold, both) if b])
    it_warm = np.mean([r.inner_iters for r, b in zip(warm, both) if b])
    print(f"DR iterations where both converge: cold {it_cold:.1f}, warm {it_warm:.1f}; "
          f"converged cold {ok_c.sum()}, warm {ok_w.sum()} of 64", flush=True)
    assert it_warm < it_cold
