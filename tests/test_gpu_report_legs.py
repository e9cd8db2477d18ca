"""GPU parity of the report's experiment legs that report.py times.

* Padding (Methodology; Results, Table 1): the same FP16 problems on copies
  zero-padded to tile multiples in M, N and K.  The padded launch has the
  unpadded one's tiles, iterations and schedule, and zero rows, columns and
  k-values contribute exact zeros, so the output's top-left M x N block must
  equal the unpadded output bit for bit, the padding region must be zero, and
  both are within the FP16 tolerance of the oracle.
* The data-parallel + one-tile Stream-K split (dp_tiles = T - T mod g, so only
  the last partial wave's tiles are split): the device trace equals the
  simulator run on the resolved launch, every MAC iteration runs once, and
  the full output matches the oracle.
"""
import pytest
import torch

import paper_2407_00044_amd as sk
from gpu_util import as64, dev, gpu, make_inputs, oracle, rel_err
from oracle import schedule as sch

pytestmark = gpu

TILE = (256, 128)
BK = 64


def cdiv(a, b):
    return -(-a // b)


@pytest.mark.parametrize("M,N,K", [(1920, 2000, 2000), (480, 512, 512), (1000, 700, 1000)])
def test_padded_leg_equals_unpadded_bitwise(M, N, K):
    print(f"case padded {M}x{N}x{K} f16 {TILE}", flush=True)
    A, B = make_inputs(M, N, K, "f16", False, True, seed=71)
    Mp, Np, Kp = cdiv(M, TILE[0]) * TILE[0], cdiv(N, TILE[1]) * TILE[1], cdiv(K, BK) * BK
    Ap = torch.zeros((Mp, Kp), dtype=torch.float16, device=dev())
    Ap[:M, :K] = A.view
    Bt = torch.zeros((Np, Kp), dtype=torch.float16, device=dev())   # B column-major
    Bt[:N, :K] = B.view.t()
    cfg = sk.Config(tile=TILE, mode="hybrid")
    p_u = sk.plan([(M, N, K)], torch.float16, cfg)
    p_p = sk.plan([(Mp, Np, Kp)], torch.float16, cfg)
    for key in ("T", "S", "g", "q", "rho", "group_m", "max_iters"):
        assert p_u[key] == p_p[key], key
    o = sk.gemm(A.view, B.view, config=cfg)
    op = sk.gemm(Ap, Bt.t(), config=cfg)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    assert torch.equal(op[:M, :N], o)
    assert not op[M:, :].any() and not op[:, N:].any()
    assert rel_err(as64(o), oracle(A, B, M, N, K)) <= 1e-4


@pytest.mark.parametrize("M,N,K,g", [(1920, 2000, 2000, 48), (1000, 700, 900, 13),
                                     (3840, 4096, 4096, 256)])
def test_one_tile_hybrid_trace_and_full_oracle(M, N, K, g):
    print(f"case one-tile hybrid {M}x{N}x{K} f16 {TILE} g={g}", flush=True)
    T = cdiv(M, TILE[0]) * cdiv(N, TILE[1])
    cfg = sk.Config(tile=TILE, mode="hybrid", num_cu=g, dp_tiles=T - T % g, min_iters=1)
    plan = sk.plan([(M, N, K)], torch.float16, cfg)
    assert plan["T"] == T and plan["S"] == T % g and 0 < plan["S"] < T
    A, B = make_inputs(M, N, K, "f16", False, True, seed=72)
    out, segs, cover = sk.gemm_debug(A.view, B.view, config=cfg)
    lp = sk.launch_params([(M, N, K)], torch.float16, cfg)
    _, sim = sch.simulate([(M, N, K)], TILE[0], TILE[1], BK, **lp)
    assert segs == [s.as_tuple() for s in sim]
    I = plan["max_iters"]
    assert torch.equal(cover[:T, :I], torch.ones((T, I), dtype=torch.int32))
    assert rel_err(as64(out), oracle(A, B, M, N, K)) <= 1e-4
    # the same launch without debug hooks gives the same bits
    again = sk.gemm(A.view, B.view, config=cfg)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    assert torch.equal(again, out)
