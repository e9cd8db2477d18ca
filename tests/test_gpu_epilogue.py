"""Fused linear-layer epilogue (bias per output column, then ReLU / GELU /
SiLU, all in FP32 on the finished FP32 sum) against the oracle: the FP64
product of the same rounded inputs, then the FP64 epilogue.

* every schedule (all Stream-K with split tiles, hybrid, data-parallel) on a
  ragged shape, FP32 / BF16 / e4m3 inputs: within the input type's tolerance;
* small integers with an integer bias and ReLU: bit-exact;
* 16-bit outputs equal the round-to-nearest-even of the FP32 output;
* alpha, beta * C_in, a bias and SiLU together; an activation without bias;
* grouped launches (a bias per problem, some None), MXFP8 and the
  allocation-free entry point;
* the full 3840x4096x4096 BF16 product with a bias and GELU.
"""
import numpy as np
import pytest
import torch

import paper_2407_00044_amd as sk
from gpu_util import TOL, as64, dev, gpu, make_inputs, oracle, rel_err
from oracle import gemm as og
from paper_2407_00044_amd import synth

pytestmark = gpu

ACTS = ["none", "relu", "gelu", "silu"]


def bias_vec(N, seed, scale=4.0):
    b64 = synth.uniform((1, N), seed)[0] * scale
    return torch.from_numpy(b64).float().to(dev())


def run(A, B, cfg, bias, act, out_dtype=torch.float32, **kw):
    out = sk.gemm(A.view, B.view, kw.pop("C", None), scale_a=A.scale, scale_b=B.scale,
                  bias=bias, activation=act, out_dtype=out_dtype, config=cfg, **kw)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    return out


def expect(A, B, M, N, K, bias, act, **kw):
    b = None if bias is None else bias.cpu().numpy().astype(np.float64)
    return og.epilogue(oracle(A, B, M, N, K, **kw), b, act)


def configs(tile):
    return {"sk": sk.Config(tile=tile, mode="sk", num_cu=23, min_iters=1),
            "hybrid": sk.Config(tile=tile, mode="hybrid", num_cu=5, min_iters=1),
            "dp": sk.Config(tile=tile, mode="dp")}


@pytest.mark.parametrize("dtype,tile", [("f32", (128, 128)), ("bf16", (128, 128)),
                                        ("bf16", (256, 128)), ("e4m3", (256, 128))])
@pytest.mark.parametrize("act", ACTS)
@pytest.mark.parametrize("mode", ["sk", "hybrid", "dp"])
def test_epilogue_parity(dtype, tile, act, mode):
    M, N, K = 300, 260, 520
    print(f"case epilogue {dtype} {tile} {act} {mode} {M}x{N}x{K}", flush=True)
    A, B = make_inputs(M, N, K, dtype, False, True, seed=41)
    bias = bias_vec(N, 42)
    cfg = configs(tile)[mode]
    if mode != "dp":
        assert sk.plan([(M, N, K)], A.view.dtype, cfg)["S"] > 0
    got = run(A, B, cfg, bias, act)
    assert rel_err(as64(got), expect(A, B, M, N, K, bias, act)) <= TOL[dtype]


def test_epilogue_integers_bit_exact_with_relu():
    M, N, K = 390, 200, 384
    print(f"case epilogue integers relu {M}x{N}x{K}", flush=True)
    A, B = make_inputs(M, N, K, "bf16", False, True, seed=43, dist="int")
    bias = torch.from_numpy(np.random.default_rng(44).integers(-60, 61, N).astype(np.float32)
                            ).to(dev())
    for mode, cfg in configs((128, 128)).items():
        got = run(A, B, cfg, bias, "relu")
        exact = expect(A, B, M, N, K, bias, "relu")
        assert np.max(np.abs(exact)) < 2 ** 24
        assert np.array_equal(as64(got), exact), mode
        assert (as64(got) == 0).any() and (as64(got) > 0).any()   # both sides of ReLU


@pytest.mark.parametrize("act", ["relu", "gelu", "silu"])
def test_epilogue_16bit_outputs_are_rne_of_fp32(act):
    M, N, K = 300, 200, 256
    print(f"case epilogue 16-bit outputs {act}", flush=True)
    A, B = make_inputs(M, N, K, "bf16", False, True, seed=45)
    bias = bias_vec(N, 46)
    cfg = sk.Config(tile=(128, 128), mode="sk", num_cu=9, min_iters=1)
    f32 = run(A, B, cfg, bias, act)
    for od in (torch.bfloat16, torch.float16):
        o = run(A, B, cfg, bias, act, out_dtype=od)
        assert torch.equal(o.cpu(), f32.cpu().to(od))


def test_epilogue_alpha_beta_cin_bias_silu_and_activation_without_bias():
    M, N, K = 333, 277, 640
    print(f"case epilogue alpha/beta/C_in silu {M}x{N}x{K}", flush=True)
    A, B = make_inputs(M, N, K, "f16", False, True, seed=47)
    cin64 = synth.uniform((M, N), 48)
    Cin = torch.from_numpy(cin64).float().to(dev())
    bias = bias_vec(N, 49)
    cfg = sk.Config(tile=(128, 128), mode="hybrid", num_cu=7, min_iters=1)
    got = run(A, B, cfg, bias, "silu", C=Cin.clone(), alpha=0.75, beta=-1.5)
    ref = expect(A, B, M, N, K, bias, "silu", alpha=0.75, beta=-1.5, cin=cin64)
    assert rel_err(as64(got), ref) <= TOL["f16"]
    got = run(A, B, cfg, None, "gelu")
    assert rel_err(as64(got), expect(A, B, M, N, K, None, "gelu")) <= TOL["f16"]


def test_epilogue_grouped_bias_per_problem():
    shapes = [(700, 300, 512), (64, 1000, 256), (257, 129, 1024), (1, 64, 64), (500, 500, 128)]
    print(f"case epilogue grouped {shapes}", flush=True)
    ops, biases = [], []
    for i, (M, N, K) in enumerate(shapes):
        A, B = make_inputs(M, N, K, "bf16", False, True, seed=50 + i, dist="normal")
        ops.append((A, B, torch.full((M, N), float("nan"), device=dev())))
        biases.append(None if i == 2 else bias_vec(N, 60 + i))
    for mode in ("sk", "hybrid", "dp"):
        cfg = sk.Config(tile=(128, 128), mode=mode, num_cu=11, min_iters=1)
        gg = sk.GroupedGemm([(A.view, B.view, out) for A, B, out in ops], config=cfg,
                            biases=biases, activation="gelu")
        gg.run()
        torch.cuda.synchronize()
        assert sk.check_device_error(workspace=gg.workspace) == 0
        if mode != "dp":
            assert gg.info()["S"] > 0
        for (A, B, out), (M, N, K), b in zip(ops, shapes, biases):
            ref = expect(A, B, M, N, K, b, "gelu")
            assert rel_err(as64(out), ref) <= TOL["bf16"], (mode, M, N, K)


def test_epilogue_mxfp8_and_noalloc():
    M, N, K = 300, 260, 512
    print(f"case epilogue mxfp8 + noalloc {M}x{N}x{K}", flush=True)
    qa, sa = synth.mx_quantize(synth.normal((M, K), 70))
    qb, sb = synth.mx_quantize(synth.normal((N, K), 71))
    bias = bias_vec(N, 72)
    cfg = sk.Config(tile=(128, 128), mode="hybrid", num_cu=9, min_iters=1)
    got = sk.gemm_mx(qa.to(dev()), qb.to(dev()).t(), torch.from_numpy(sa).to(dev()),
                     torch.from_numpy(sb).to(dev()), bias=bias, activation="silu", config=cfg)
    torch.cuda.synchronize()
    ref = og.epilogue(og.gemm_mx(M, N, K, synth.codes(qa), K, sa, K // 32, synth.codes(qb), K,
                                 sb, K // 32), bias.cpu().numpy().astype(np.float64), "silu")
    assert rel_err(as64(got), ref) <= 1e-4
    A, B = make_inputs(M, N, K, "bf16", False, True, seed=73)
    out = torch.empty((M, N), device=dev())
    sk.gemm_noalloc(A.view, B.view, out=out, bias=bias, activation="relu", config=cfg)
    torch.cuda.synchronize()
    assert sk.check_noalloc_error() == 0
    assert rel_err(as64(out), expect(A, B, M, N, K, bias, "relu")) <= TOL["bf16"]


def test_epilogue_headline_shape_full_matrix():
    M, N, K = 3840, 4096, 4096
    print(f"case epilogue bf16 {M}x{N}x{K} 256x256 gelu, full matrix", flush=True)
    A, B = make_inputs(M, N, K, "bf16", False, True, seed=74)
    bias = bias_vec(N, 75)
    ref = expect(A, B, M, N, K, bias, "gelu")
    for mode in ("hybrid", "dp"):
        got = run(A, B, sk.Config(tile=(256, 256), mode=mode), bias, "gelu")
        assert rel_err(as64(got), ref) <= TOL["bf16"], mode
