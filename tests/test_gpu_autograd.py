"""Differentiable linear layer Y = X W^T with the hand-written Stream-K
backward (dX = dY W, dW = dY^T X through the same kernels at transposed
layouts).

* finite differences: L(X, W) = sum(dY * (X W^T)) is linear in X and in W,
  so FP64 central differences of L computed with the oracle GEMM reproduce
  the analytic gradients up to rounding; the GPU backward is compared with
  those at 64x48x32 (X [64,32], W [48,32]);
* a BF16 layer whose three products all split tiles, against the oracle
  gradient;
* full size BF16: X [8192,4096], W [11008,4096], dY [8192,11008]; every
  element of Y, dX and dW against the oracle, and the BF16 gradients equal
  the round-to-nearest-even of the FP32 kernel outputs."""
import numpy as np
import pytest
import torch

import paper_2407_00044_amd as sk
from gpu_util import as64, dev, gpu
from oracle import gemm as og
from paper_2407_00044_amd import synth

pytestmark = gpu


def loss64(X, W, dY):
    """L = sum(dY * (X W^T)) in FP64 through the oracle GEMM."""
    Y = og.gemm_dense(X, W.T)
    return float(np.sum(dY * Y))


def fd_grad(X, W, dY, wrt):
    """Central differences of L with respect to X or W."""
    P = X if wrt == "X" else W
    G = np.zeros_like(P)
    for idx in np.ndindex(P.shape):
        h = 2.0 ** -10 * max(1.0, abs(P[idx]))
        old = P[idx]
        P[idx] = old + h
        lp = loss64(X, W, dY)
        P[idx] = old - h
        lm = loss64(X, W, dY)
        P[idx] = old
        G[idx] = (lp - lm) / (2 * h)
    return G


# (dtype, workgroups, grid floor): FP32 on 2 workgroups with the floor off
# splits the backward's products (dX: K = 48, dW: K = 64, i.e. 2 iterations
# of 32 each, one per workgroup), so the partial/finish fixup runs under the
# finite-difference check; BF16 iterations hold 64 K-values, so at this size
# every product is one iteration per tile and nothing can split (the split
# BF16 backward is checked against the oracle gradient below).
FD_CASES = [(torch.float32, 2, 1), (torch.float32, 7, 0), (torch.bfloat16, 7, 0)]


@pytest.mark.parametrize("dtype,g,mi", FD_CASES)
def test_finite_differences_64x48x32(dtype, g, mi):
    M, N, K = 64, 48, 32
    name = "f32" if dtype == torch.float32 else "bf16"
    X = synth.round_to(synth.normal((M, K), 41), name)
    W = synth.round_to(synth.normal((N, K), 42), name)
    dY = synth.round_to(synth.normal((M, N), 43), name)
    X64, W64, dY64 = (t.double().numpy().copy() for t in (X, W, dY))
    gX_fd = fd_grad(X64, W64, dY64, "X")
    gW_fd = fd_grad(X64, W64, dY64, "W")
    # the analytic FP64 gradients agree with the differences (L is linear)
    assert og.rel_frobenius(og.gemm_dense(dY64, W64), gX_fd) < 1e-10
    assert og.rel_frobenius(og.gemm_dense(dY64.T, X64), gW_fd) < 1e-10

    Xg = X.to(dev()).requires_grad_(True)
    Wg = W.to(dev()).requires_grad_(True)
    cfg = sk.Config(tile=(128, 128), mode="sk", num_cu=g, min_iters=mi)
    if mi == 1:
        for shape in [(M, K, N), (N, K, M)]:            # dX, dW
            p = sk.plan([shape], dtype, cfg)
            assert p["S"] > 0 and p["g"] == 2 and p["W"] == 2
            segs = sk.schedule([shape], dtype, cfg)
            assert [s[7] for s in segs] == [1, 2]         # FINISH on 0, PARTIAL on 1
    Y = sk.linear(Xg, Wg, cfg, cfg, cfg)
    Y.backward(dY.to(dev()))
    tol = 1e-5 if dtype == torch.float32 else 1e-4
    # parity on FP32 kernel outputs at the backward's layouts
    gx32 = sk.gemm(dY.to(dev()), Wg.detach(), config=cfg)
    gw32 = sk.gemm(dY.to(dev()).t(), Xg.detach(), config=cfg)
    assert og.rel_frobenius(as64(gx32), gX_fd) < tol
    assert og.rel_frobenius(as64(gw32), gW_fd) < tol
    assert torch.equal(Xg.grad.cpu(), gx32.cpu().to(dtype))
    assert torch.equal(Wg.grad.cpu(), gw32.cpu().to(dtype))
    y32 = sk.gemm(Xg.detach(), Wg.detach().t(), config=cfg)
    assert og.rel_frobenius(as64(y32), og.gemm_dense(X64, W64.T)) < tol
    assert torch.equal(Y.detach().cpu(), y32.cpu().to(dtype))


def test_bf16_backward_split_against_oracle_gradient():
    # X [320, 384], W [448, 384]: forward 320x448x384 (6 iterations per
    # tile), dX 320x384x448 (7), dW 448x384x320 (5) on 128x128 tiles and 5
    # workgroups without a grid floor: every product splits tiles; the
    # gradients against the oracle's FP64 products of the same rounded inputs
    M, N, K = 320, 448, 384
    X = synth.round_to(synth.normal((M, K), 44), "bf16")
    W = synth.round_to(synth.normal((N, K), 45), "bf16")
    dY = synth.round_to(synth.normal((M, N), 46), "bf16")
    cfg = sk.Config(tile=(128, 128), mode="sk", num_cu=5, min_iters=1)
    for shape in [(M, N, K), (M, K, N), (N, K, M)]:
        assert sk.plan([shape], torch.bfloat16, cfg)["S"] > 0
        assert any(s[7] == 1 for s in sk.schedule([shape], torch.bfloat16, cfg))
    Xg = X.to(dev()).requires_grad_(True)
    Wg = W.to(dev()).requires_grad_(True)
    Y = sk.linear(Xg, Wg, cfg, cfg, cfg)
    Y.backward(dY.to(dev()))
    X64, W64, dY64 = (t.double().numpy() for t in (X, W, dY))
    y32 = sk.gemm(Xg.detach(), Wg.detach().t(), config=cfg)
    gx32 = sk.gemm(dY.to(dev()), Wg.detach(), config=cfg)
    gw32 = sk.gemm(dY.to(dev()).t(), Xg.detach(), config=cfg)
    assert og.rel_frobenius(as64(y32), og.gemm_dense(X64, W64.T)) <= 1e-4
    assert og.rel_frobenius(as64(gx32), og.gemm_dense(dY64, W64)) <= 1e-4
    assert og.rel_frobenius(as64(gw32), og.gemm_dense(dY64.T, X64)) <= 1e-4
    assert torch.equal(Xg.grad.cpu(), gx32.cpu().to(torch.bfloat16))
    assert torch.equal(Wg.grad.cpu(), gw32.cpu().to(torch.bfloat16))
    assert torch.equal(Y.detach().cpu(), y32.cpu().to(torch.bfloat16))


def test_full_size_bf16_linear_every_element():
    M, N, K = 8192, 11008, 4096
    X = synth.round_to(synth.normal((M, K), 4), "bf16")
    W = synth.round_to(synth.normal((N, K), 5), "bf16")
    dY = synth.round_to(synth.normal((M, N), 40), "bf16")
    Xg = X.to(dev()).requires_grad_(True)
    Wg = W.to(dev()).requires_grad_(True)
    dYg = dY.to(dev())
    cf = sk.Config(tile=(256, 256), mode="hybrid")
    cdx = sk.Config(tile=(256, 128), mode="hybrid")
    cdw = sk.Config(tile=(256, 128), mode="hybrid")
    Y = sk.linear(Xg, Wg, cf, cdx, cdw)
    Y.backward(dYg)
    y32 = sk.gemm(Xg.detach(), Wg.detach().t(), config=cf)
    dx32 = sk.gemm(dYg, Wg.detach(), config=cdx)
    dw32 = sk.gemm(dYg.t(), Xg.detach(), config=cdw)
    torch.cuda.synchronize()
    assert torch.equal(Y.detach(), y32.to(torch.bfloat16))
    assert torch.equal(Xg.grad, dx32.to(torch.bfloat16))
    assert torch.equal(Wg.grad, dw32.to(torch.bfloat16))
    X64 = X.double().numpy()
    W64 = W.double().numpy()
    dY64 = dY.double().numpy()
    ref = og.gemm(M, N, K, X64, K, False, W64, K, True)       # Y = X W^T
    assert og.rel_frobenius(as64(y32), ref) <= 1e-4
    del ref
    ref = og.gemm(M, K, N, dY64, N, False, W64, K, False)     # dX = dY W
    assert og.rel_frobenius(as64(dx32), ref) <= 1e-4
    del ref
    ref = og.gemm(N, K, M, dY64, N, True, X64, K, False)      # dW = dY^T X
    assert og.rel_frobenius(as64(dw32), ref) <= 1e-4
