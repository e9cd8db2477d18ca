"""Operand packing (sk_transpose) and the packed backward of the linear layer.

* sk_transpose against torch's transposed copy, bit for bit: 1-, 2- and
  4-byte elements (random bit patterns, NaN codes included), ragged shapes
  around the 64 x 64 tile, padded leading dimensions, and a base pointer off
  the 8-byte grid (the element-wise path);
* K-contiguous copies of M- and N-major operands give the same GEMM as the
  operands as laid out, bit for bit: both read the same values into the
  same matrix-core lanes in the same order;
* the linear layer's backward with packed operands (the automatic rule
  packs at this size) against the oracle's FP64 products and, bit for bit,
  against the backward on the operands as laid out."""
import pytest
import torch

import paper_2407_00044_amd as sk
from gpu_util import as64, dev, gpu
from oracle import gemm as og
from paper_2407_00044_amd import synth

pytestmark = gpu

BITS = {torch.uint8: torch.uint8, torch.float8_e4m3fn: torch.uint8,
        torch.float16: torch.int16, torch.bfloat16: torch.int16, torch.float32: torch.int32}


def random_bits(rows, cols, dtype, seed):
    """rows x cols tensor of `dtype` whose bytes are uniform random."""
    eb = torch.tensor([], dtype=dtype).element_size()
    g = torch.Generator().manual_seed(seed)
    raw = torch.randint(0, 256, (rows, cols * eb), generator=g, dtype=torch.uint8)
    return raw.view(dtype).to(dev())


def same_bits(a, b):
    return torch.equal(a.view(BITS[a.dtype]), b.view(BITS[b.dtype]))


SHAPES = [(1, 1), (1, 70), (70, 1), (63, 65), (64, 64), (130, 257), (1000, 3000)]


@pytest.mark.parametrize("dtype", [torch.uint8, torch.float8_e4m3fn, torch.bfloat16,
                                   torch.float16, torch.float32])
def test_transpose_bit_exact(dtype):
    for i, (r, c) in enumerate(SHAPES):
        print(f"case transpose {dtype} {r}x{c}", flush=True)
        t = random_bits(r, c, dtype, 10 + i)
        assert same_bits(sk.transpose(t), t.t().contiguous())
        # padded leading dimension, and a view starting one element in (its
        # rows are then off the 8-byte grid: the element-wise path)
        big = random_bits(r, c + 9, dtype, 50 + i)
        for view in (big[:, :c], big[:, 1:c + 1]):
            assert same_bits(sk.transpose(view), view.t().contiguous())
    torch.cuda.synchronize()


def test_transpose_empty_and_layout_checks():
    for r, c in [(0, 5), (5, 0)]:
        u = sk.transpose(torch.empty((r, c), dtype=torch.bfloat16, device=dev()))
        assert tuple(u.shape) == (c, r)
    with pytest.raises(ValueError):
        sk.transpose(torch.empty((8, 6), dtype=torch.bfloat16, device=dev()).t())


@pytest.mark.parametrize("dtype", ["bf16", "e4m3"])
def test_k_contiguous_copies_give_the_same_gemm(dtype):
    # A M-major and B N-major (both read through transposing LDS reads), then
    # their K-contiguous copies: identical outputs, on a tile that splits
    M, N, K = 700, 900, 1000
    print(f"case packed gemm {dtype} {M}x{N}x{K}", flush=True)
    if dtype == "e4m3":
        a, _ = synth.fp8_scaled(synth.normal((M, K), 61))
        b, _ = synth.fp8_scaled(synth.normal((K, N), 62))
    else:
        a = synth.round_to(synth.normal((M, K), 61), dtype)
        b = synth.round_to(synth.normal((K, N), 62), dtype)
    A, _, _ = synth.place(a, col_major=True, device=dev())
    B, _, _ = synth.place(b, col_major=False, device=dev())
    Ak, Bk = sk.k_contiguous(A, "a"), sk.k_contiguous(B, "b")
    assert Ak.stride(1) == 1 and Bk.stride(0) == 1
    for tile in [(256, 256), (256, 128)]:
        cfg = sk.Config(tile=tile, mode="sk", num_cu=64, min_iters=1)
        assert sk.plan([(M, N, K)], A.dtype, cfg)["S"] > 0
        got = sk.gemm(A, B, config=cfg)
        packed = sk.gemm(Ak, Bk, config=cfg)
        torch.cuda.synchronize()
        assert torch.equal(got, packed), tile
        assert torch.equal(sk.gemm(A, B, config=cfg, pack=True), packed), tile
    ref = og.gemm_dense(a.float().double().numpy(), b.float().double().numpy())
    assert og.rel_frobenius(as64(packed), ref) <= 1e-4


def test_packed_linear_backward():
    # X [2304, 2048], W [2560, 2048]: dX 2304x2048x2560 and dW 2560x2048x2304
    # are packed by the automatic rule; their gradients equal the backward
    # on the operands as laid out, and the oracle's products within 1e-4
    M, N, K = 2304, 2560, 2048
    assert sk.pack_pays(M, K, N, torch.bfloat16) and sk.pack_pays(N, K, M, torch.bfloat16)
    X = synth.round_to(synth.normal((M, K), 71), "bf16")
    W = synth.round_to(synth.normal((N, K), 72), "bf16")
    dY = synth.round_to(synth.normal((M, N), 73), "bf16")
    cfg = sk.Config(tile=(256, 128), mode="hybrid")
    grads = {}
    for pack in ("auto", False):
        print(f"case packed backward pack={pack}", flush=True)
        Xg = X.to(dev()).requires_grad_(True)
        Wg = W.to(dev()).requires_grad_(True)
        sk.linear(Xg, Wg, cfg, cfg, cfg, pack=pack).backward(dY.to(dev()))
        grads[pack] = (Xg.grad.clone(), Wg.grad.clone())
    torch.cuda.synchronize()
    assert torch.equal(grads["auto"][0], grads[False][0])
    assert torch.equal(grads["auto"][1], grads[False][1])
    gx32 = sk.gemm(dY.to(dev()), sk.k_contiguous(W.to(dev()), "b"), config=cfg)
    gw32 = sk.gemm(sk.k_contiguous(dY.to(dev()).t(), "a"), sk.k_contiguous(X.to(dev()), "b"),
                   config=cfg)
    assert torch.equal(grads["auto"][0], gx32.to(torch.bfloat16))
    assert torch.equal(grads["auto"][1], gw32.to(torch.bfloat16))
    X64, W64, dY64 = (t.double().numpy() for t in (X, W, dY))
    assert og.rel_frobenius(as64(gx32), og.gemm_dense(dY64, W64)) <= 1e-4
    assert og.rel_frobenius(as64(gw32), og.gemm_dense(dY64.T, X64)) <= 1e-4
