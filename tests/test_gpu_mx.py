"""MXFP8 (OCP MX block scaling: e4m3 elements, an E8M0 scale per 32 K-values
of each row of A and column of B) through sk_gemm_mx against the oracle's
MX product (block scales applied exactly in FP64, then the plain product).

* random normal inputs quantised per block, every schedule and both tiles,
  ragged M and N: within 1e-4 relative Frobenius error (FP32 accumulation);
* small-integer elements with scales 2^-1 .. 2^2: every product and partial
  sum is exact in FP32, so the result equals the oracle bit for bit;
* the headline shape on the full matrix, alpha and an in-place beta * C;
* scale-row padding (bytes past K/32) holds NaN codes, which must never be
  read.
"""
import numpy as np
import pytest
import torch

import paper_2407_00044_amd as sk
from gpu_util import as64, dev, gpu, rel_err
from oracle import gemm as og
from paper_2407_00044_amd import synth

pytestmark = gpu


def mx_inputs(M, N, K, seed, dist="normal"):
    if dist == "normal":
        a64 = synth.normal((M, K), seed)
        b64 = synth.normal((N, K), seed + 1)            # B^T: column j of B is row j
        qa, sa = synth.mx_quantize(a64)
        qb, sb = synth.mx_quantize(b64)
    else:
        rng = np.random.default_rng(seed)
        qa = torch.from_numpy(rng.integers(-4, 5, size=(M, K)).astype(np.float64)).to(
            torch.float8_e4m3fn)
        qb = torch.from_numpy(rng.integers(-4, 5, size=(N, K)).astype(np.float64)).to(
            torch.float8_e4m3fn)
        sa = rng.integers(126, 130, size=(M, K // 32)).astype(np.uint8)
        sb = rng.integers(126, 130, size=(N, K // 32)).astype(np.uint8)
    # scale rows padded to a multiple of 4 bytes plus 4, the padding NaN (255)
    lds = (K // 32 + 3) // 4 * 4 + 4
    pa = np.full((M, lds), 255, np.uint8)
    pa[:, :K // 32] = sa
    pb = np.full((N, lds), 255, np.uint8)
    pb[:, :K // 32] = sb
    A = qa.to(dev())
    B = qb.to(dev()).t()                                 # K x N, column-major
    SA = torch.from_numpy(pa).to(dev())
    SB = torch.from_numpy(pb).to(dev())
    ref = lambda alpha=1.0, beta=0.0, cin=None: og.gemm_mx(  # noqa: E731
        M, N, K, synth.codes(qa), K, pa, lds, synth.codes(qb), K, pb, lds, alpha, beta, cin)
    return A, B, SA, SB, ref


@pytest.mark.parametrize("M,N,K", [(300, 260, 512), (1000, 700, 1024), (64, 2000, 2048)])
@pytest.mark.parametrize("tile", [(128, 128), (256, 128)])
@pytest.mark.parametrize("mode", ["sk", "hybrid", "dp", "auto"])
def test_mx_parity(M, N, K, tile, mode):
    print(f"case mx {M}x{N}x{K} {tile} {mode}", flush=True)
    A, B, SA, SB, ref = mx_inputs(M, N, K, seed=81)
    cfg = sk.Config(tile=tile, mode=mode, num_cu=256, min_iters=1 if mode == "sk" else 0)
    out = sk.gemm_mx(A, B, SA, SB, config=cfg)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    assert rel_err(as64(out), ref()) <= 1e-4


@pytest.mark.parametrize("tile", [(128, 128), (256, 128)])
def test_mx_integers_bit_exact(tile):
    M, N, K = 520, 390, 1024
    print(f"case mx integers {M}x{N}x{K} {tile}", flush=True)
    A, B, SA, SB, ref = mx_inputs(M, N, K, seed=82, dist="int")
    for mode in ("sk", "hybrid"):
        cfg = sk.Config(tile=tile, mode=mode, num_cu=256, min_iters=1)
        out = sk.gemm_mx(A, B, SA, SB, config=cfg)
        torch.cuda.synchronize()
        exact = ref()
        assert np.max(np.abs(exact)) < 2 ** 24
        assert np.array_equal(as64(out), exact)


def test_mx_headline_shape_full_matrix_alpha_beta():
    M, N, K = 3840, 4096, 4096
    print(f"case mx {M}x{N}x{K} 256x128 hybrid alpha/beta", flush=True)
    A, B, SA, SB, ref = mx_inputs(M, N, K, seed=83)
    cin = torch.linspace(-1, 1, M * N, device=dev()).reshape(M, N)
    cfg = sk.Config(tile=(256, 128), mode="hybrid")
    out = sk.gemm_mx(A, B, SA, SB, cin.clone(), alpha=2.0, beta=0.5, config=cfg)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    expect = ref(2.0, 0.5, cin.cpu().numpy().astype(np.float64))
    assert rel_err(as64(out), expect) <= 1e-4


GROUP = [(300, 260, 512), (64, 1000, 1024), (1000, 129, 256), (1, 64, 128), (513, 700, 384)]


def grouped_mx_inputs(shapes, seed, dist="normal"):
    probs, scales, refs = [], [], []
    for i, (M, N, K) in enumerate(shapes):
        A, B, SA, SB, ref = mx_inputs(M, N, K, seed + 10 * i, dist)
        out = torch.full((M, N), float("nan"), device=dev())
        probs.append((A, B, out))
        scales.append((SA, SB))
        refs.append(ref)
    return probs, scales, refs


@pytest.mark.parametrize("tile", [(128, 128), (256, 128)])
@pytest.mark.parametrize("mode", ["sk", "hybrid", "dp", "auto"])
def test_mx_grouped_parity(tile, mode):
    print(f"case mx grouped {tile} {mode}", flush=True)
    probs, scales, refs = grouped_mx_inputs(GROUP, 91)
    cfg = sk.Config(tile=tile, mode=mode, num_cu=23, min_iters=1 if mode == "sk" else 0)
    gg = sk.GroupedGemm(probs, config=cfg, mx_scales=scales)
    if mode in ("sk", "hybrid"):
        assert gg.info()["S"] > 0
    gg.run()
    torch.cuda.synchronize()
    assert sk.check_device_error(workspace=gg.workspace) == 0
    for (A, B, out), ref in zip(probs, refs):
        assert rel_err(as64(out), ref()) <= 1e-4, tuple(out.shape)


def test_mx_grouped_integers_bit_exact_and_graph_replays():
    print("case mx grouped integers + graph", flush=True)
    probs, scales, refs = grouped_mx_inputs(GROUP, 92, dist="int")
    cfg = sk.Config(tile=(256, 128), mode="hybrid", num_cu=37, min_iters=1)
    gg = sk.GroupedGemm(probs, config=cfg, mx_scales=scales)
    gg.run()
    torch.cuda.synchronize()
    first = []
    for (A, B, out), ref in zip(probs, refs):
        assert np.array_equal(as64(out), ref())
        first.append(out.clone())
    g = gg.capture()
    for r in range(3):
        for _, _, out in probs:
            out.fill_(float("nan"))              # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (_, _, out), f in zip(probs, first):
            assert torch.equal(out, f), f"replay {r} differs"
