"""MXFP8 with e5m2 elements (OCP MX block scaling: an E8M0 scale per 32
K-values of each row of A and column of B) through sk_gemm_mx against the
oracle's MX product (block scales applied exactly in FP64, then the plain
product).

* random normal inputs quantised per block into e5m2, every schedule and
  both tiles, ragged M and N: within 1e-4 relative Frobenius error (FP32
  accumulation);
* elements from -6 .. 6 (all e5m2 values) with scales 2^-1 .. 2^2: every
  product and partial sum is exact in FP32, so the result equals the oracle
  bit for bit, and differs from the same codes read as e4m3;
* the headline shape on the full matrix, alpha and an in-place beta * C;
* a grouped launch of uneven problems, against the oracle and bitwise
  across graph replays;
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

INTS = np.array([-6, -4, -3, -2, -1, 0, 1, 2, 3, 4, 6], dtype=np.float64)


def e5_inputs(M, N, K, seed, dist="normal"):
    if dist == "normal":
        qa, sa = synth.mx_quantize(synth.normal((M, K), seed), elem="e5m2")
        qb, sb = synth.mx_quantize(synth.normal((N, K), seed + 1), elem="e5m2")  # B^T rows
    else:
        rng = np.random.default_rng(seed)
        qa = torch.from_numpy(rng.choice(INTS, size=(M, K))).to(torch.float8_e5m2)
        qb = torch.from_numpy(rng.choice(INTS, size=(N, K))).to(torch.float8_e5m2)
        sa = rng.integers(126, 130, size=(M, K // 32)).astype(np.uint8)
        sb = rng.integers(126, 130, size=(N, K // 32)).astype(np.uint8)
    lds = (K // 32 + 3) // 4 * 4 + 4          # padded scale rows, padding NaN (255)
    pa = np.full((M, lds), 255, np.uint8)
    pa[:, :K // 32] = sa
    pb = np.full((N, lds), 255, np.uint8)
    pb[:, :K // 32] = sb
    ca, cb = qa.view(torch.uint8).numpy(), qb.view(torch.uint8).numpy()
    A = qa.to(dev())
    B = qb.to(dev()).t()                                 # K x N, column-major
    SA = torch.from_numpy(pa).to(dev())
    SB = torch.from_numpy(pb).to(dev())
    ref = lambda alpha=1.0, beta=0.0, cin=None, elem="e5m2": og.gemm_mx(  # noqa: E731
        M, N, K, ca, K, pa, lds, cb, K, pb, lds, alpha, beta, cin, elem=elem)
    return A, B, SA, SB, ref


@pytest.mark.parametrize("M,N,K", [(300, 260, 512), (1000, 700, 1024), (64, 2000, 2048)])
@pytest.mark.parametrize("tile", [(128, 128), (256, 128)])
@pytest.mark.parametrize("mode", ["sk", "hybrid", "dp"])
def test_mx8e5_parity(M, N, K, tile, mode):
    print(f"case mx8 e5m2 {M}x{N}x{K} {tile} {mode}", flush=True)
    A, B, SA, SB, ref = e5_inputs(M, N, K, seed=381)
    cfg = sk.Config(tile=tile, mode=mode, num_cu=256, min_iters=1 if mode == "sk" else 0)
    out = sk.gemm_mx(A, B, SA, SB, config=cfg)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    assert rel_err(as64(out), ref()) <= 1e-4


@pytest.mark.parametrize("tile", [(128, 128), (256, 128)])
def test_mx8e5_integers_bit_exact(tile):
    M, N, K = 520, 390, 1024
    print(f"case mx8 e5m2 integers {M}x{N}x{K} {tile}", flush=True)
    A, B, SA, SB, ref = e5_inputs(M, N, K, seed=382, dist="int")
    exact = ref()
    assert np.max(np.abs(exact)) < 2 ** 24
    # the same bytes read as e4m3 give another product: the format is honoured
    assert not np.array_equal(exact, ref(elem="e4m3"))
    for mode in ("sk", "hybrid"):
        cfg = sk.Config(tile=tile, mode=mode, num_cu=256, min_iters=1)
        out = sk.gemm_mx(A, B, SA, SB, config=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(as64(out), exact), mode


def test_mx8e5_headline_shape_full_matrix_alpha_beta():
    M, N, K = 3840, 4096, 4096
    print(f"case mx8 e5m2 {M}x{N}x{K} 256x128 hybrid alpha/beta", flush=True)
    A, B, SA, SB, ref = e5_inputs(M, N, K, seed=383)
    cin = torch.linspace(-1, 1, M * N, device=dev()).reshape(M, N)
    cfg = sk.Config(tile=(256, 128), mode="hybrid")
    out = sk.gemm_mx(A, B, SA, SB, cin.clone(), alpha=2.0, beta=0.5, config=cfg)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    expect = ref(2.0, 0.5, cin.cpu().numpy().astype(np.float64))
    assert rel_err(as64(out), expect) <= 1e-4


GROUP = [(300, 260, 512), (64, 1000, 1024), (1000, 129, 256), (1, 64, 128), (513, 700, 384)]


@pytest.mark.parametrize("mode", ["sk", "hybrid"])
def test_mx8e5_grouped_parity_and_replays(mode):
    print(f"case mx8 e5m2 grouped {mode}", flush=True)
    probs, scales, refs = [], [], []
    for i, (M, N, K) in enumerate(GROUP):
        A, B, SA, SB, ref = e5_inputs(M, N, K, 390 + 10 * i)
        probs.append((A, B, torch.full((M, N), float("nan"), device=dev())))
        scales.append((SA, SB))
        refs.append(ref)
    cfg = sk.Config(tile=(128, 128), mode=mode, num_cu=23, min_iters=1 if mode == "sk" else 0)
    gg = sk.GroupedGemm(probs, config=cfg, mx_scales=scales)
    assert gg.info()["S"] > 0 and gg.info()["dtype_ab"] == sk.api.MX8_CODES[torch.float8_e5m2]
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
