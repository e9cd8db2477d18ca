"""OCP e5m2 inputs with per-tensor scales (the FP8 gradient format) through
sk_gemm against the oracle's FP64 product of the decoded codes.

* amax-scaled normal inputs, every operand layout and every tile of the
  8-bit menu, Stream-K and the two-tile hybrid, ragged M, N and K tails:
  within 1e-4 relative Frobenius error (FP32 accumulation);
* small-integer codes: every product and partial sum is exact in FP32, so
  the result equals the oracle bit for bit, and differs from the same bytes
  read as e4m3;
* a grouped launch of uneven problems in mixed layouts.
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


def e5_operands(M, N, K, seed, a_col, b_col, dist="normal"):
    if dist == "normal":
        a, sa = synth.fp8_scaled(synth.normal((M, K), seed), elem="e5m2")
        b, sb = synth.fp8_scaled(synth.normal((K, N), seed + 1), elem="e5m2")
    else:
        rng = np.random.default_rng(seed)
        a = torch.from_numpy(rng.choice(INTS, size=(M, K))).to(torch.float8_e5m2)
        b = torch.from_numpy(rng.choice(INTS, size=(K, N))).to(torch.float8_e5m2)
        sa = sb = 1.0
    A, _, _ = synth.place(a, col_major=a_col, device=dev())
    B, _, _ = synth.place(b, col_major=b_col, device=dev())
    dec = lambda t, f: f(t.view(torch.uint8).numpy())   # noqa: E731
    ref = og.gemm_dense(dec(a, og.decode_e5m2), dec(b, og.decode_e5m2)) * (sa * sb)
    alt = og.gemm_dense(dec(a, og.decode_e4m3fn), dec(b, og.decode_e4m3fn)) * (sa * sb)
    return A, B, sa, sb, ref, alt


LAYOUTS = {"rc": (False, True), "rr": (False, False), "cr": (True, False), "cc": (True, True)}


@pytest.mark.parametrize("lay", list(LAYOUTS))
@pytest.mark.parametrize("tile", [(256, 256), (256, 128), (128, 128), (64, 128)])
@pytest.mark.parametrize("mode", ["sk", "hybrid"])
def test_e5m2_parity(lay, tile, mode):
    M, N, K = 700, 520, 1000
    print(f"case e5m2 {lay} {tile} {mode} {M}x{N}x{K}", flush=True)
    A, B, sa, sb, ref, _ = e5_operands(M, N, K, 481, *LAYOUTS[lay])
    cfg = sk.Config(tile=tile, mode=mode, num_cu=64, min_iters=1)
    out = sk.gemm(A, B, scale_a=sa, scale_b=sb, config=cfg)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    assert rel_err(as64(out), ref) <= 1e-4


@pytest.mark.parametrize("lay", ["rc", "cr"])
def test_e5m2_integers_bit_exact(lay):
    M, N, K = 520, 390, 1024
    print(f"case e5m2 integers {lay}", flush=True)
    A, B, _, _, ref, alt = e5_operands(M, N, K, 482, *LAYOUTS[lay], dist="int")
    assert np.max(np.abs(ref)) < 2 ** 24 and not np.array_equal(ref, alt)
    for tile in [(256, 128), (128, 128)]:
        cfg = sk.Config(tile=tile, mode="hybrid", num_cu=256, min_iters=1)
        out = sk.gemm(A, B, config=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(as64(out), ref), tile


def test_e5m2_grouped():
    print("case e5m2 grouped", flush=True)
    shapes = [(300, 260, 512), (64, 1000, 1024), (1000, 129, 256), (513, 700, 384)]
    probs, refs = [], []
    for i, (M, N, K) in enumerate(shapes):
        A, B, sa, sb, ref, _ = e5_operands(M, N, K, 490 + 10 * i, False, True)
        probs.append((A, B, torch.full((M, N), float("nan"), device=dev())))
        refs.append((ref, sa * sb))
    cfg = sk.Config(tile=(128, 128), mode="hybrid", num_cu=23, min_iters=1)
    gg = sk.GroupedGemm(probs, config=cfg)
    assert gg.info()["S"] > 0
    gg.run()
    torch.cuda.synchronize()
    assert sk.check_device_error(workspace=gg.workspace) == 0
    for (_, _, out), (ref, s) in zip(probs, refs):
        assert rel_err(as64(out) * s, ref) <= 1e-4, tuple(out.shape)
