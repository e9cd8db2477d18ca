"""Grouped GEMM through sk_grouped_prepare / sk_gemm_grouped: one persistent
launch over many uneven problems, captured into a HIP graph.

Workload of record: 48 FP8-e4m3 problems, M log-uniform in [16, 4096],
N in {1024, 2048, 4096}, K in {2048, 4096, 8192}, N(0,1) entries amax-scaled
to the e4m3 range with per-tensor scales, FP32 accumulation and output."""
import numpy as np
import pytest
import torch

import paper_2407_00044_amd as sk
from gpu_util import TOL, as64, dev, gpu, make_inputs, oracle, rel_err
from oracle import schedule as sch
from paper_2407_00044_amd import synth

pytestmark = gpu


def build(shapes, dtype, seed0, dist="normal", a_col=False, b_col=True):
    ops = []
    for i, (M, N, K) in enumerate(shapes):
        A, B = make_inputs(M, N, K, dtype, a_col, b_col, seed0 + i, dist)
        out = torch.full((M, N), float("nan"), device=dev())
        ops.append((A, B, out))
    return ops


def check_group(ops, cfg, rows_per_problem=None, exact=False, replays=0):
    problems = [(A.view, B.view, out) for A, B, out in ops]
    scales = [(A.scale, B.scale) for A, B, _ in ops]
    gg = sk.GroupedGemm(problems, config=cfg, scales=scales)
    gg.run()
    torch.cuda.synchronize()
    assert sk.check_device_error(workspace=gg.workspace) == 0
    first = [out.clone() for _, _, out in ops]
    for i, (A, B, out) in enumerate(ops):
        M, N = out.shape
        K = A.view.shape[1]
        rows = None
        if rows_per_problem and M > rows_per_problem:
            rows = np.unique(np.random.default_rng(i).integers(0, M, rows_per_problem))
        ref = oracle(A, B, M, N, K, rows=rows)
        got = as64(out) if rows is None else as64(out)[rows]
        if exact:
            assert np.array_equal(got, ref), i
        else:
            assert rel_err(got, ref) <= TOL[A.dtype], (i, rel_err(got, ref))
    if replays:
        g = gg.capture()
        for r in range(replays):
            for _, _, out in ops:
                out.fill_(float("nan"))          # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for o, f in zip([out for _, _, out in ops], first):
                assert torch.equal(o, f), f"replay {r} differs"
    return gg


def test_grouped_schedule_matches_simulator():
    # host schedule and the device trace of the launch both equal the
    # simulator run on the launch parameters the library resolved
    shapes = synth.grouped_shapes()
    for tile in [(64, 128), (128, 128), (256, 128)]:
        for mode in ["hybrid", "sk", "auto"]:
            cfg = sk.Config(tile=tile, mode=mode, num_cu=256)
            lp = sk.launch_params(shapes, torch.float8_e4m3fn, cfg)
            _, sim = sch.simulate(shapes, tile[0], tile[1], 128, **lp)
            want = [s.as_tuple() for s in sim]
            assert sk.schedule(shapes, torch.float8_e4m3fn, cfg) == want


@pytest.mark.parametrize("mode", ["hybrid", "sk", "auto"])
def test_grouped_device_trace_matches_simulator(mode):
    # the kernel's grouped tile lookup (binary search over the problems'
    # iteration and tile offsets) against the simulator, segment by segment,
    # on a 12-problem subset of the FP8 workload plus ragged and empty
    # problems; every MAC iteration runs exactly once
    shapes = synth.grouped_shapes()[:12] + [(0, 64, 64), (129, 257, 100), (16, 1024, 300)]
    print(f"case grouped trace {len(shapes)} problems mode={mode}", flush=True)
    ops = build(shapes, "e4m3", 900)
    problems = [(A.view, B.view, out) for A, B, out in ops]
    scales = [(A.scale, B.scale) for A, B, _ in ops]
    cfg = sk.Config(tile=(128, 128), mode=mode, num_cu=256)
    gg = sk.GroupedGemm(problems, config=cfg, scales=scales)
    segs, cover = gg.run_debug()
    lp = sk.launch_params(shapes, torch.float8_e4m3fn, cfg)
    _, sim = sch.simulate(shapes, 128, 128, 128, **lp)
    assert segs == [s.as_tuple() for s in sim]
    T = int(gg.plan.T)
    iters = [max(1, -(-K // 128)) for p in lp["order"] for (M, N, K) in [shapes[p]]
             for _ in range(-(-M // 128) * -(-N // 128) if M and N else 0)]
    assert len(iters) == T
    for t, I in enumerate(iters):
        assert torch.equal(cover[t, :I], torch.ones(I, dtype=torch.int32)), t
    for i, (A, B, out) in enumerate(ops):
        M, N = out.shape
        if M and N:
            ref = oracle(A, B, M, N, A.view.shape[1])
            assert rel_err(as64(out), ref) <= TOL["e4m3"], i


@pytest.mark.parametrize("dtype", ["bf16", "e4m3", "f32"])
def test_grouped_small_full_oracle(dtype):
    shapes = [(16, 128, 256), (300, 200, 520), (1, 64, 64), (129, 257, 100), (0, 64, 64),
              (64, 0, 64), (200, 64, 0), (513, 130, 1000)]
    tile = (128, 128)
    for mode in ["sk", "hybrid", "dp"]:
        ops = build(shapes, dtype, 100)
        check_group(ops, sk.Config(tile=tile, mode=mode, num_cu=37))


def test_grouped_integer_bit_exact_and_graph_replays():
    shapes = [(100, 300, 700), (64, 128, 2000), (257, 64, 129), (16, 1024, 300)]
    ops = build(shapes, "e4m3", 200, dist="int")
    check_group(ops, sk.Config(tile=(64, 128), mode="sk", num_cu=256), exact=True, replays=10)


def test_c5_fp8_grouped_48_problems_graph():
    shapes = synth.grouped_shapes()
    ops = build(shapes, "e4m3", 500)
    # every element of all 48 products against the oracle
    gg = check_group(ops, sk.Config(tile=(128, 128), mode="hybrid", num_cu=256), replays=10)
    info = gg.info()
    assert info["nprobs"] == 48 and info["T"] > 0


@pytest.mark.parametrize("dtype", ["bf16", "e4m3"])
@pytest.mark.parametrize("a_col,b_col", [(True, False), (False, False), (True, True)])
def test_grouped_m_n_major_layouts(dtype, a_col, b_col):
    # one grouped launch whose operands are M- or N-contiguous (copied into
    # LDS as k-rows and read back transposed), ragged in every dimension
    shapes = [(300, 200, 520), (129, 257, 1000), (513, 130, 96), (64, 384, 777)]
    for tile in [(128, 128), (256, 128)]:
        for mode in ["sk", "hybrid"]:
            ops = build(shapes, dtype, 700, a_col=a_col, b_col=b_col)
            check_group(ops, sk.Config(tile=tile, mode=mode, num_cu=29))
