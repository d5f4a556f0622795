"""Small end-to-end run of the learned warm start on the GPU: generate solves
with the plain batched method, train the network with the project's kernels,
warm-start held-out problems, and check that every warm-started solve reaches
the 1e-4 residual as often as the cold starts (the fallback keeps the cold point
when the warm one is worse), and that, where both converge, the warm starts
do not need more DR iterations than cold starts on average."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_learned_warm_start_small():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_02642_amd import learned as L
    from paper_2603_02642_amd import nrto
    opt = L.dr_options(max_admm=200)
    X, Y, ok = L.generate(192, chunk=192, opt=opt, log=lambda *a: None)
    assert ok.sum() >= 24
    net, norm = L.train(X[ok], Y[ok], epochs=30, batch=64, log=lambda *a: None)
    probs = L.problems("heldout", 0, 32)
    ctx = nrto.Context(probs, opt)
    ctx.linearize()
    cold = ctx.solve()
    feats = torch.from_numpy(L.features(probs)).cuda()
    pred = net.infer(feats)
    acc, res = ctx.warm_start(pred)
    warm = ctx.solve(warm=True)
    ok_c = np.array([r.kkt <= 1e-4 for r in cold])
    ok_w = np.array([r.kkt <= 1e-4 for r in warm])
    assert ok_w.sum() >= ok_c.sum() - 1
    both = ok_c & ok_w
    assert both.sum() >= 4
    it_cold = np.mean([r.inner_iters for r, b in zip(cold, both) if b])
    it_warm = np.mean([r.inner_iters for r, b in zip(warm, both) if b])
    assert it_warm <= 1.05 * it_cold
