"""The allocation-free entry point sk_gemm_noalloc against sk_gemm.

Both run the same kernels with the same plan, so their outputs must agree
bit for bit; each is also within the oracle tolerance of its input type.
Two calls in a row share the library's static scratch array, the second
with a smaller problem (and a different split point and workgroup count),
then a launch on the largest plan the array holds; a plan beyond it is
rejected on the host before anything is launched."""
import pytest
import torch

import paper_2407_00044_amd as sk
from gpu_util import TOL, as64, gpu, make_inputs, oracle, rel_err, run
from paper_2407_00044_amd import _abi

pytestmark = gpu


def noalloc(A, B, cfg, beta=0.0, C=None):
    out = torch.empty((A.view.shape[0], B.view.shape[1]), dtype=torch.float32,
                      device=A.view.device)
    sk.gemm_noalloc(A.view, B.view, C, beta=beta, out=out if C is None else C,
                    scale_a=A.scale, scale_b=B.scale, config=cfg)
    torch.cuda.synchronize()
    assert sk.check_noalloc_error() == 0
    return out if C is None else C


def test_noalloc_matches_sk_gemm_on_two_calls_and_rejects_oversize():
    # call 1: every tile split (all Stream-K over 256 workgroups), BF16
    M, N, K = 1000, 1100, 2000
    A, B = make_inputs(M, N, K, "bf16", False, True, seed=61)
    cfg = sk.Config(tile=(128, 128), mode="sk", num_cu=256, min_iters=1)
    assert sk.plan([(M, N, K)], torch.bfloat16, cfg)["S"] > 0
    got = noalloc(A, B, cfg)
    ref = run(A, B, cfg)
    assert torch.equal(got, ref)
    assert rel_err(as64(got), oracle(A, B, M, N, K)) <= TOL["bf16"]

    # call 2: smaller, FP32, fewer workgroups and a different split point
    M2, N2, K2 = 300, 260, 520
    A2, B2 = make_inputs(M2, N2, K2, "f32", True, False, seed=62)
    cfg2 = sk.Config(tile=(128, 128), mode="hybrid", num_cu=23, min_iters=1)
    p2 = sk.plan([(M2, N2, K2)], torch.float32, cfg2)
    assert p2["S"] > 0 and p2["g"] == 23
    got2 = noalloc(A2, B2, cfg2)
    ref2 = run(A2, B2, cfg2)
    assert torch.equal(got2, ref2)
    assert rel_err(as64(got2), oracle(A2, B2, M2, N2, K2)) <= TOL["f32"]

    # the largest plan the scratch holds: 256 workgroups of 256x256 partial
    # tiles, with beta * C_in in place
    M3, N3, K3 = 1024, 1280, 4096
    A3, B3 = make_inputs(M3, N3, K3, "bf16", False, True, seed=63)
    cfg3 = sk.Config(tile=(256, 256), mode="sk", num_cu=256, min_iters=1)
    p3 = sk.plan([(M3, N3, K3)], torch.bfloat16, cfg3)
    assert p3["g"] == 256 and p3["S"] > 0
    assert p3["workspace_bytes"] == _abi_scratch_bytes()
    cin = torch.linspace(-1, 1, M3 * N3, device=A3.view.device).reshape(M3, N3)
    got3 = noalloc(A3, B3, cfg3, beta=0.5, C=cin.clone())
    ref3 = run(A3, B3, cfg3, beta=0.5, C=cin.clone())
    assert torch.equal(got3, ref3)
    exp3 = oracle(A3, B3, M3, N3, K3, beta=0.5, cin=cin.cpu().numpy().astype("float64"))
    assert rel_err(as64(got3), exp3) <= TOL["bf16"]

    # beyond the scratch: 512 workgroups of 256x256 partial tiles
    cfg4 = sk.Config(tile=(256, 256), mode="sk", num_cu=0, wg_per_cu=2, min_iters=1)
    with pytest.raises(_abi.StreamKError) as e:
        sk.gemm_noalloc(A3.view, B3.view, config=cfg4)
    assert e.value.status == _abi.SK_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert sk.check_noalloc_error() == 0


def _abi_scratch_bytes():
    return 16640 + 256 * 256 * 256 * 4
