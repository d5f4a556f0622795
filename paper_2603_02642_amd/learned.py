"""Learned warm start for batched NRTO-DR (quadrotor, T = 50, 10 obstacles).

Pipeline (all numerics in libnrto: solves, network forward/backward/Adam,
warm-start reconstruction and the fallback test):
  1. generate: solve the first successive-linearisation SOCP of seeded
     training problems with the plain batched method (cold start) and keep
     (features, du, p~, pi) of the converged ones;
  2. train: standardise features and targets, then Adam steps of the GELU MLP
     64 -> 256 x 4 -> 1400 on the GPU;
  3. warm-started solves: network inference -> nrto_warm_start (DR fixed-point
     reconstruction, cold fallback when the warm KKT residual is worse) ->
     nrto_solve_socp continuing from that state.

Usage:
  python -m paper_2603_02642_amd.learned train --n-train 20000 --out PATH.npz
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

from . import nrto  # noqa: E402

# output: du (T*nu = 200), p~ (n_g = 600), pi (n_g) of the quadrotor SOCP; the gains
# are not predicted (the warm start keeps the cold point's gains)
WIDTHS = [64, 256, 256, 256, 256, 1400]


def dr_options(**kw):
    base = dict(method=nrto.NRTO_DR, precision=nrto.NRTO_FP64, max_admm=200, max_inner=100,
                check_every=1, rho=50.0, sigma_s=100.0, cold_init=1, sigma_adapt=1, sigma_thr=2.0,
                eps_kkt=1e-4)
    base.update(kw)
    return nrto.default_options(**base)


def problems(split, start, count):
    return [synth.config5_instance(i, split) for i in range(start, start + count)]


def features(probs):
    return np.stack([synth.mlp_features(p) for p in probs]).astype(np.float32)


def solve_batch(probs, opt, stream=None):
    """Cold batched solve; returns (targets (n x 1400): du, p~, pi; reports)."""
    ctx = nrto.Context(probs, opt, stream=stream)
    ctx.linearize()
    rep = ctx.solve()
    rows = []
    for i in range(ctx.n):
        s = ctx.solution(i)
        rows.append(np.concatenate([s["du"], s["pt"], s["pi"]]))
    ctx.close()
    return np.array(rows, dtype=np.float32), rep


def generate(n, chunk=2048, split="train", opt=None, log=print):
    opt = opt or dr_options()
    X, Y, ok = [], [], []
    t0 = time.perf_counter()
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        probs = problems(split, s, m)
        tgt, rep = solve_batch(probs, opt)
        X.append(features(probs))
        Y.append(tgt)
        ok.append(np.array([r.kkt <= 1e-4 for r in rep]))
        log(f"generate {s + m}/{n}: {np.mean(ok[-1]) * 100:.1f}% converged, "
            f"mean admm {np.mean([r.admm_iters for r in rep]):.1f}, {time.perf_counter() - t0:.1f}s")
    return np.concatenate(X), np.concatenate(Y), np.concatenate(ok)


def train(X, Y, epochs=40, batch=256, lr=1e-3, seed=0, log=print):
    import torch
    net = nrto.WarmStartNet(WIDTHS, max(batch, 4096), seed=seed)
    xm, xs = X.mean(0), X.std(0) + 1e-6
    ym, ys = Y.mean(0), Y.std(0) + 1e-6
    net.set_norm(xm, xs, ym, ys)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.from_numpy(Y).cuda()
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        last = 0.0
        for b in range(0, n - batch + 1, batch):
            idx = perm[b:b + batch]
            want = b + 2 * batch > n
            last = net.train_step(Xd[idx].contiguous(), Yd[idx].contiguous(), lr, want_loss=want)
        if ep % 5 == 0 or ep == epochs - 1:
            log(f"epoch {ep}: loss {last:.4f}")
    return net, (xm, xs, ym, ys)


def save(net, norm, path):
    params = net.get_params()
    flat = {f"W{l}": W for l, (W, b) in enumerate(params)}
    flat.update({f"b{l}": b for l, (W, b) in enumerate(params)})
    xm, xs, ym, ys = norm
    np.savez_compressed(path, xm=xm, xs=xs, ym=ym, ys=ys, widths=np.array(WIDTHS), gains=np.array(0), **flat)


def rows_have_gains(path) -> bool:
    """Whether the network at path predicts K (rows du, K, p~, pi) or not (du, p~, pi)."""
    d = np.load(path, allow_pickle=False)
    return bool(d["gains"]) if "gains" in d.files else True


def load_net(path, max_batch=4096):
    d = np.load(path, allow_pickle=False)
    widths = [int(w) for w in d["widths"]]
    net = nrto.WarmStartNet(widths, max_batch)
    net.set_params([[d[f"W{l}"], d[f"b{l}"]] for l in range(len(widths) - 1)])
    net.set_norm(d["xm"], d["xs"], d["ym"], d["ys"])
    return net


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train"])
    ap.add_argument("--n-train", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    torch.cuda.synchronize()
    X, Y, ok = generate(a.n_train)
    print(f"training on {int(ok.sum())} converged solves", flush=True)
    net, norm = train(X[ok], Y[ok], epochs=a.epochs)
    save(net, norm, a.out)
    print("saved", a.out, flush=True)


if __name__ == "__main__":
    main()
