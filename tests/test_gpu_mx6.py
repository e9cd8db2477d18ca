"""MXFP6 (OCP MX: six-bit E2M3 or E3M2 elements packed little-endian, an
E8M0 scale per 32 K-values of each row of A and column of B) through
sk_gemm_mx against the oracle's MX product (block scales applied exactly in
FP64, then the plain product).

* random normal inputs quantised per block, both formats, every schedule
  and both tiles, ragged M and N, several iterations: within 1e-4 relative
  Frobenius error (FP32 accumulation);
* elements from 0, +-1, +-2, +-3, +-4, +-6 with scales 2^-1 .. 2^2: every
  product and partial sum is exact in FP32, so the result equals the oracle
  bit for bit;
* the headline shape on the full matrix, alpha and an in-place beta * C, and
  the fused epilogue;
* scale-row padding (bytes past K/32) holds NaN codes, which must never be
  read;
* a grouped launch of five uneven problems per format, against the oracle
  and bitwise across graph replays.
"""
import numpy as np
import pytest
import torch

import paper_2407_00044_amd as sk
from gpu_util import as64, dev, gpu, rel_err
from oracle import gemm as og
from paper_2407_00044_amd import synth

pytestmark = gpu

# codes of 0, 1, 2, 3, 4, 6 and their negatives (exact small values)
INT_CODES = {"e2m3": np.array([0, 8, 16, 20, 24, 28, 40, 48, 52, 56, 60]),
             "e3m2": np.array([0, 12, 16, 18, 20, 22, 44, 48, 50, 52, 54])}


def mx6_inputs(M, N, K, fmt, seed, dist="normal"):
    if dist == "normal":
        pa, sa = synth.mx6_quantize(synth.normal((M, K), seed), fmt)
        pb, sb = synth.mx6_quantize(synth.normal((N, K), seed + 1), fmt)   # B^T rows
    else:
        rng = np.random.default_rng(seed)
        pa = synth.pack_fp6(rng.choice(INT_CODES[fmt], size=(M, K)))
        pb = synth.pack_fp6(rng.choice(INT_CODES[fmt], size=(N, K)))
        sa = rng.integers(126, 130, size=(M, K // 32)).astype(np.uint8)
        sb = rng.integers(126, 130, size=(N, K // 32)).astype(np.uint8)
    lds = (K // 32 + 3) // 4 * 4 + 4          # padded scale rows, padding NaN (255)
    qa = np.full((M, lds), 255, np.uint8)
    qa[:, :K // 32] = sa
    qb = np.full((N, lds), 255, np.uint8)
    qb[:, :K // 32] = sb
    A = torch.from_numpy(pa).to(dev())                       # M x 3K/4, row-major
    B = torch.from_numpy(pb).to(dev()).t()                   # 3K/4 x N, column-major
    SA = torch.from_numpy(qa).to(dev())
    SB = torch.from_numpy(qb).to(dev())
    ref = lambda alpha=1.0, beta=0.0, cin=None: og.gemm_mx(  # noqa: E731
        M, N, K, pa, K, qa, lds, pb, K, qb, lds, alpha, beta, cin, elem=fmt)
    return A, B, SA, SB, ref


@pytest.mark.parametrize("fmt", ["e2m3", "e3m2"])
@pytest.mark.parametrize("M,N,K", [(300, 260, 512), (1000, 700, 1024), (64, 2000, 1152)])
@pytest.mark.parametrize("tile", [(128, 128), (256, 128)])
@pytest.mark.parametrize("mode", ["sk", "hybrid", "dp"])
def test_mx6_parity(fmt, M, N, K, tile, mode):
    print(f"case mx6 {fmt} {M}x{N}x{K} {tile} {mode}", flush=True)
    A, B, SA, SB, ref = mx6_inputs(M, N, K, fmt, seed=281)
    cfg = sk.Config(tile=tile, mode=mode, num_cu=256, min_iters=1 if mode == "sk" else 0)
    out = sk.gemm_mx6(A, B, SA, SB, fmt=fmt, config=cfg)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    assert rel_err(as64(out), ref()) <= 1e-4


@pytest.mark.parametrize("fmt", ["e2m3", "e3m2"])
@pytest.mark.parametrize("tile", [(128, 128), (256, 128)])
def test_mx6_exact_values_bit_exact(fmt, tile):
    M, N, K = 520, 390, 1024
    print(f"case mx6 exact values {fmt} {M}x{N}x{K} {tile}", flush=True)
    A, B, SA, SB, ref = mx6_inputs(M, N, K, fmt, seed=282, dist="int")
    exact = ref()
    assert np.max(np.abs(exact)) < 2 ** 22
    for mode in ("sk", "hybrid"):
        cfg = sk.Config(tile=tile, mode=mode, num_cu=256, min_iters=1)
        out = sk.gemm_mx6(A, B, SA, SB, fmt=fmt, config=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(as64(out), exact), mode


def test_mx6_headline_shape_full_matrix_alpha_beta():
    M, N, K = 3840, 4096, 4096
    print(f"case mx6 {M}x{N}x{K} 256x128 hybrid alpha/beta", flush=True)
    A, B, SA, SB, ref = mx6_inputs(M, N, K, "e2m3", seed=283)
    cin = torch.linspace(-1, 1, M * N, device=dev()).reshape(M, N)
    cfg = sk.Config(tile=(256, 128), mode="hybrid")
    out = sk.gemm_mx6(A, B, SA, SB, cin.clone(), alpha=2.0, beta=0.5, config=cfg)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    expect = ref(2.0, 0.5, cin.cpu().numpy().astype(np.float64))
    assert rel_err(as64(out), expect) <= 1e-4


def test_mx6_fused_epilogue():
    M, N, K = 300, 260, 512
    print(f"case mx6 bias + silu {M}x{N}x{K}", flush=True)
    A, B, SA, SB, ref = mx6_inputs(M, N, K, "e3m2", seed=284)
    bias = torch.from_numpy(synth.uniform((1, N), 285)[0] * 4).float().to(dev())
    out = sk.gemm_mx6(A, B, SA, SB, fmt="e3m2", bias=bias, activation="silu",
                      config=sk.Config(tile=(128, 128), mode="hybrid", num_cu=9, min_iters=1))
    torch.cuda.synchronize()
    expect = og.epilogue(ref(), bias.cpu().numpy().astype(np.float64), "silu")
    assert rel_err(as64(out), expect) <= 1e-4


GROUP = [(300, 260, 512), (64, 1000, 1024), (1000, 129, 256), (1, 64, 256), (513, 700, 768)]


@pytest.mark.parametrize("fmt", ["e2m3", "e3m2"])
@pytest.mark.parametrize("mode", ["sk", "hybrid"])
def test_mx6_grouped_parity_and_replays(fmt, mode):
    print(f"case mx6 grouped {fmt} {mode}", flush=True)
    probs, scales, refs = [], [], []
    for i, (M, N, K) in enumerate(GROUP):
        A, B, SA, SB, ref = mx6_inputs(M, N, K, fmt, 290 + 10 * i)
        probs.append((A, B, torch.full((M, N), float("nan"), device=dev())))
        scales.append((SA, SB))
        refs.append(ref)
    cfg = sk.Config(tile=(128, 128), mode=mode, num_cu=23, min_iters=1 if mode == "sk" else 0)
    gg = sk.GroupedGemm(probs, config=cfg, mx_scales=scales, mx_format=fmt)
    assert gg.info()["S"] > 0 and gg.info()["dtype_ab"] == sk.api.MX6_FORMATS[fmt]
    gg.run()
    torch.cuda.synchronize()
    assert sk.check_device_error(workspace=gg.workspace) == 0
    first = []
    for (A, B, out), ref in zip(probs, refs):
        assert rel_err(as64(out), ref()) <= 1e-4, tuple(out.shape)
        first.append(out.clone())
    g = gg.capture()
    for r in range(2):
        for _, _, out in probs:
            out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (_, _, out), f in zip(probs, first):
            assert torch.equal(out, f), f"replay {r} differs"
