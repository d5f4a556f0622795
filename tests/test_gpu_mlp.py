"""GPU checks of the warm-start network kernels: the BF16 matrix-core GEMM
(fragment layouts, ragged edges, strided operands) against an exact product
of the bf16-rounded inputs, the network's forward pass and gradients against
the FP64 reference MLP on the same parameters (with and without its bfloat16
operand rounding), and the Adam kernel against the reference Adam."""
import numpy as np
import pytest

import synth
from oracle import mlp

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _bf16_bits(x):
    """Round-to-nearest-even float32 -> bf16 bit patterns (test-side marshalling)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def _bits_to_f64(b):
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K,trans_a,trans_b", [(64, 64, 32, False, False), (77, 45, 50, False, True),
                                                  (130, 200, 96, True, False), (5, 3800, 256, False, True),
                                                  (136, 72, 104, True, False), (200, 136, 88, False, True),
                                                  (256, 1400, 256, False, True)])
def test_gemm_bf16_matches_exact_product(M, N, K, trans_a, trans_b):
    torch = _torch()
    from paper_2603_02642_amd import nrto
    a = 2 * synth.uniform(1, M * K) - 1
    b = 2 * synth.uniform(2, K * N) - 1
    Ab = _bf16_bits(a.reshape(M, K) if not trans_a else a.reshape(M, K).T.copy())
    Bb = _bf16_bits(b.reshape(K, N) if not trans_b else b.reshape(K, N).T.copy())
    sam, sak = (K, 1) if not trans_a else (1, M)
    sbk, sbn = (N, 1) if not trans_b else (1, K)
    ref = _bits_to_f64(Ab) if not trans_a else _bits_to_f64(Ab).T
    refb = _bits_to_f64(Bb) if not trans_b else _bits_to_f64(Bb).T
    C_ref = ref @ refb
    At = torch.from_numpy(Ab.view(np.int16)).cuda()
    Bt = torch.from_numpy(Bb.view(np.int16)).cuda()
    Ct = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    nrto.gemm_bf16(At, sam, sak, Bt, sbk, sbn, M, N, K, Ct)
    C = Ct.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(C - C_ref)) <= 1e-5 * max(1.0, np.max(np.abs(C_ref)))


def _net_case(torch, widths, B):
    from paper_2603_02642_amd import nrto
    net = nrto.WarmStartNet(widths, B, seed=7)
    X = (2 * synth.uniform(3, B * widths[0]) - 1).reshape(B, widths[0]).astype(np.float32)
    T = synth.uniform(4, B * widths[-1]).reshape(B, widths[-1]).astype(np.float32)
    return net, X, T


@pytest.mark.parametrize("widths,B", [([64, 256, 256, 256, 256, 1400], 64), ([64, 256, 256, 256, 256, 3800], 32)])
def test_forward_and_gradients_match_reference(widths, B):
    """Against the FP64 reference with the GEMM operands rounded to bfloat16 as
    the matrix cores see them (1e-3 relative), and against the exact FP64
    reference (bf16 operand rounding only, 2e-2)."""
    torch = _torch()
    net, X, T = _net_case(torch, widths, B)
    params = [[W.astype(np.float64), b.astype(np.float64)] for W, b in net.get_params()]
    for l in range(len(params)):           # non-zero biases exercise the bias paths
        params[l][1] = 0.05 * (2 * synth.uniform(50 + l, params[l][1].size) - 1)
    net.set_params(params)
    params = [[W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)]
              for W, b in params]
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T).cuda()
    X64, T64 = X.astype(np.float64), T.astype(np.float64)
    Y = net.infer(Xd).cpu().numpy().astype(np.float64)
    Yq, _, _ = mlp.forward(params, X64, rnd=mlp.round_bf16)
    Yr, _, _ = mlp.forward(params, X64)
    assert np.linalg.norm(Y - Yq) <= 1e-3 * np.linalg.norm(Yq)
    assert np.linalg.norm(Y - Yr) <= 2e-2 * np.linalg.norm(Yr)
    grads, loss = net.gradients(Xd, Td)
    lq, gq = mlp.loss_and_grads(params, X64, T64, rnd=mlp.round_bf16)
    lr, gr = mlp.loss_and_grads(params, X64, T64)
    assert abs(loss - lq) <= 1e-3 * lq
    assert abs(loss - lr) <= 2e-2 * lr
    for l in range(len(params)):
        for i in range(2):
            g = grads[l][i].astype(np.float64)
            assert np.linalg.norm(g - gq[l][i]) <= 1e-3 * np.linalg.norm(gq[l][i]) + 1e-12, (l, i)
            assert np.linalg.norm(g - gr[l][i]) <= 3e-2 * np.linalg.norm(gr[l][i]) + 1e-12, (l, i)


def test_adam_steps_match_reference_elementwise():
    """Two Adam steps of the device optimizer against the reference Adam applied
    to the same (device) gradients from the same parameters."""
    torch = _torch()
    widths = [64, 256, 256, 1400]
    net, X, T = _net_case(torch, widths, 64)
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T).cuda()
    ref = [[W.astype(np.float64), b.astype(np.float64)] for W, b in net.get_params()]
    # the device runs Adam with the float32 values of its constants (1 - 0.999 in
    # float32 is off by 1.3e-5 relative); the reference takes the same values
    f32 = lambda v: float(np.float32(v))
    lr = f32(1e-3)
    opt = mlp.Adam(ref, lr=lr, b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8))
    for step in range(2):
        g, _ = net.gradients(Xd, Td)
        net.train_step(Xd, Td, 1e-3, want_loss=False)
        opt.step(ref, [[gw.astype(np.float64), gb.astype(np.float64)] for gw, gb in g])
        got = net.get_params()
        for l in range(len(ref)):
            for i in range(2):
                a = got[l][i].astype(np.float64)
                d = np.abs(a - ref[l][i])
                assert np.all(d <= 1e-6 * np.abs(ref[l][i]) + 1e-6 * lr), (step, l, i, float(d.max()))
        ref = [[W.astype(np.float64), b.astype(np.float64)] for W, b in got]   # continue from the device's values


def test_training_reduces_loss():
    torch = _torch()
    widths = [64, 256, 256, 256, 256, 64]
    net, X, T = _net_case(torch, widths, 256)
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(np.tanh(X @ (synth.uniform(9, 64 * 64).reshape(64, 64) - 0.5)).astype(np.float32)).cuda()
    l0 = net.train_step(Xd, Td, 1e-3)
    for _ in range(200):
        l1 = net.train_step(Xd, Td, 1e-3, want_loss=False)
    l1 = net.train_step(Xd, Td, 1e-3)
    assert l1 < 0.2 * l0
