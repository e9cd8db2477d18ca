"""GPU schedule and fixup checks through sk_gemm_debug.

* the segments the workgroups actually ran equal the oracle's simulator;
* every MAC iteration of every tile ran exactly once;
* results are bitwise identical across repeats, with contributors delayed
  before publishing, and with hardware workgroups mapped to logical ids in
  reverse (fixup ordering stress).
"""
import numpy as np
import pytest
import torch

import paper_2407_00044_amd as sk
from gpu_util import as64, dev, gpu, make_inputs, oracle, rel_err, run
from oracle import schedule as sch

pytestmark = gpu

BK = {"f32": 32, "f16": 64, "bf16": 64, "e4m3": 128}

# (M, N, K, dtype, tile, mode, g, min_iters): min_iters = 1 keeps all g
# workgroups (many contributors per tile); 0 applies the automatic floor
CASES = [
    (512, 512, 512, "f32", (128, 128), "sk", 256, 1),
    (384, 384, 128, "f32", (128, 128), "sk", 4, 1),
    (384, 384, 128, "f32", (128, 128), "hybrid", 4, 1),
    (1000, 700, 900, "bf16", (256, 128), "hybrid", 13, 1),
    (1000, 700, 900, "bf16", (128, 128), "sk", 256, 1),
    (480, 512, 512, "f16", (256, 128), "sk", 120, 1),
    (700, 300, 2000, "e4m3", (64, 128), "hybrid", 64, 1),
    (640, 640, 300, "bf16", (128, 128), "dp", 0, 1),
    (607, 187, 3155, "bf16", (256, 128), "hybrid", 256, 0),
    (235, 2337, 528, "bf16", (128, 128), "sk", 256, 0),
    (1000, 700, 900, "f16", (128, 128), "hybrid", 256, 7),
    (1713, 1597, 14203, "bf16", (128, 128), "auto", 256, 0),
    (1000, 700, 900, "bf16", (128, 128), "auto", 256, 0),
    # persistent data-parallel rounds (odd rounds taken back to front):
    # 48 tiles on 4 workgroups = 12 rounds; on 7: 13 split tiles + 5 rounds
    (1000, 700, 900, "bf16", (128, 128), "hybrid", 4, 1),
    (1000, 700, 900, "e4m3", (128, 128), "hybrid", 7, 1),
]


@pytest.mark.parametrize("M,N,K,dtype,tile,mode,g,mi", CASES)
def test_device_trace_matches_simulator(M, N, K, dtype, tile, mode, g, mi):
    print(f"case {M}x{N}x{K} {dtype} {tile} {mode} g={g} min_iters={mi}", flush=True)
    A, B = make_inputs(M, N, K, dtype, False, True, seed=3)
    cfg = sk.Config(tile=tile, mode=mode, num_cu=g, min_iters=mi)
    out, segs, cover = sk.gemm_debug(A.view, B.view, config=cfg, scale_a=A.scale,
                                     scale_b=B.scale)
    # the simulator runs the launch the library resolved (g, S, tile
    # order, dealing rule) and derives every segment itself
    lp = sk.launch_params([(M, N, K)], A.view.dtype, cfg)
    _, sim = sch.simulate([(M, N, K)], tile[0], tile[1], BK[dtype], **lp)
    assert segs == [s.as_tuple() for s in sim]
    plan = sk.plan([(M, N, K)], A.view.dtype, cfg)
    T, I = plan["T"], plan["max_iters"]
    assert torch.equal(cover[:T, :I], torch.ones((T, I), dtype=torch.int32))
    assert rel_err(as64(out), oracle(A, B, M, N, K)) <= (1e-5 if dtype == "f32" else 1e-4)


def test_repeats_delays_and_reversed_ids_are_bitwise_identical():
    M, N, K = 512, 512, 512
    A, B = make_inputs(M, N, K, "f32", False, False, seed=1)
    cfg = sk.Config(tile=(128, 128), mode="sk", num_cu=256, min_iters=1)
    first = run(A, B, cfg)
    for _ in range(20):
        assert torch.equal(run(A, B, cfg), first)
    for delay, rev in [(2000, 0), (0, 1), (2000, 1)]:
        out, segs, cover = sk.gemm_debug(A.view, B.view, config=cfg, partial_delay=delay,
                                         reverse_ids=rev)
        assert torch.equal(out, first)


def test_bf16_many_contributors_bitwise_repeatable():
    # K long relative to the tile count: every tile split across many WGs
    M, N, K = 256, 512, 16384
    A, B = make_inputs(M, N, K, "bf16", False, True, seed=8)
    cfg = sk.Config(tile=(256, 128), mode="sk", num_cu=256, min_iters=1)
    first = run(A, B, cfg)
    assert rel_err(as64(first), oracle(A, B, M, N, K)) <= 1e-4
    for _ in range(10):
        assert torch.equal(run(A, B, cfg), first)
    out, _, _ = sk.gemm_debug(A.view, B.view, config=cfg, partial_delay=3000, reverse_ids=1)
    assert torch.equal(out, first)


def test_spin_limit_reports_timeout_without_hanging():
    # Force the bounded fixup wait to give up: a limit of one poll, with
    # contributors that sleep before publishing.  Every wave still exits;
    # the device error word is raised and reported as a timeout.
    from paper_2407_00044_amd import _abi
    M, N, K = 512, 512, 512
    A, B = make_inputs(M, N, K, "f32", False, False, seed=1)
    cfg = sk.Config(tile=(128, 128), mode="sk", num_cu=256, spin_limit=1, min_iters=1)
    ws = sk.Workspace(dev())
    with pytest.raises(_abi.StreamKError) as e:
        sk.gemm_debug(A.view, B.view, config=cfg, partial_delay=20000, workspace=ws)
    assert e.value.status == _abi.SK_ERR_DEVICE_TIMEOUT
    # the same workspace serves the next launches without a reset: the
    # timed-out launch still advanced the workspace's epoch, so its late
    # partial tiles carry a stale tag
    for m in (1, 0):
        good = sk.gemm(A.view, B.view, config=sk.Config(tile=(128, 128), mode="sk",
                                                        num_cu=256, min_iters=m),
                       workspace=ws)
        torch.cuda.synchronize()
        assert sk.check_device_error(workspace=ws) == 0
        assert rel_err(as64(good), oracle(A, B, M, N, K)) <= 1e-5


def test_workspace_shared_across_split_points():
    # One workspace serves launches whose split points and tile counts
    # differ: a hybrid launch, then an all-Stream-K launch of 17689 tiles
    # (more tiles than the earlier launch's partial slots started after),
    # then the hybrid again; every result against the oracle.
    from paper_2407_00044_amd import _abi  # noqa: F401
    ws = sk.Workspace(dev())
    A1, B1 = make_inputs(1000, 700, 900, "bf16", False, True, seed=21)
    c_h = sk.Config(tile=(128, 128), mode="hybrid", num_cu=256, min_iters=1)
    M, N, K = 16900, 16900, 192
    A2, B2 = make_inputs(M, N, K, "bf16", False, True, seed=22)
    c_s = sk.Config(tile=(128, 128), mode="sk", num_cu=256, min_iters=1)
    p = sk.plan([(M, N, K)], torch.bfloat16, c_s)
    assert p["T"] == 17689 and p["S"] == 17689 and p["rho"] > 0
    ref1 = oracle(A1, B1, 1000, 700, 900)
    for _ in range(2):
        out = sk.gemm(A1.view, B1.view, config=c_h, workspace=ws)
        torch.cuda.synchronize()
        assert rel_err(as64(out), ref1) <= 1e-4
        out = sk.gemm(A2.view, B2.view, config=c_s, workspace=ws)
        torch.cuda.synchronize()
        assert sk.check_device_error(workspace=ws) == 0
        got = as64(out)
        ref = oracle(A2, B2, M, N, K)
        assert rel_err(got, ref) <= 1e-4
        # every tile on its own (a tile finished before its peers' partial
        # tiles arrived is off by a large fraction)
        for r0 in range(0, M, 128):
            d = got[r0:r0 + 128] - ref[r0:r0 + 128]
            rr = ref[r0:r0 + 128]
            for c0 in range(0, N, 1024):
                num = np.linalg.norm(d[:, c0:c0 + 1024])
                den = np.linalg.norm(rr[:, c0:c0 + 1024])
                assert num <= 1e-4 * den, (r0, c0)
