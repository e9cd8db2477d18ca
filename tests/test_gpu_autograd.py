"""Differentiable linear layer Y = X W^T with the hand-written Stream-K
backward (dX = dY W, dW = dY^T X through the same kernels at transposed
layouts).

* finite differences: L(X, W) = sum(dY * (X W^T)) is linear in X and in W,
  so FP64 central differences of L computed with the oracle GEMM reproduce
  the analytic gradients up to rounding; the GPU backward is compared with
  those at 64x48x32 (X [64,32], W [48,32]);
* full size BF16: X [8192,4096], W [11008,4096], dY [8192,11008]; sampled
  rows of Y, dX and dW against the oracle, and the BF16 gradients equal the
  round-to-nearest-even of the FP32 kernel outputs."""
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


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_finite_differences_64x48x32(dtype):
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
    cfg = sk.Config(tile=(128, 128), mode="sk", num_cu=7)
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


def test_full_size_bf16_linear_sampled_rows():
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
    r = np.random.default_rng(7)
    rows = np.unique(r.integers(0, M, 48))
    ref = og.gemm(M, N, K, X64, K, False, W64, K, True, rows=rows)      # Y = X W^T
    assert og.rel_frobenius(as64(y32)[rows], ref) <= 1e-4
    ref = og.gemm(M, K, N, dY64, N, False, W64, K, False, rows=rows)    # dX = dY W
    assert og.rel_frobenius(as64(dx32)[rows], ref) <= 1e-4
    rows = np.unique(r.integers(0, N, 48))
    ref = og.gemm(N, K, M, dY64, N, True, X64, K, False, rows=rows)     # dW = dY^T X
    assert og.rel_frobenius(as64(dw32)[rows], ref) <= 1e-4
