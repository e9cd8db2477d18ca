"""Autotuner on the GPU: the chosen configuration is one of the candidates,
the cache returns it unchanged on the next call, and the product it gives
matches the oracle."""
import torch

import paper_2407_00044_amd as sk
from gpu_util import TOL, as64, dev, gpu, make_inputs, oracle, rel_err
from paper_2407_00044_amd import tune

pytestmark = gpu


def _as_key(c):
    return tune.config_to_dict(c)


def test_tune_gemm_picks_a_candidate_and_caches_it(tmp_path, monkeypatch):
    monkeypatch.setenv("SK_TUNE_CACHE", str(tmp_path / "tune.json"))
    M, N, K = 700, 900, 1500
    A, B = make_inputs(M, N, K, "bf16", False, True, 11, "normal")
    report = []
    best = tune.tune_gemm(A.view, B.view, reps=3, report=report)
    cands = [_as_key(c) for c in tune.candidates([(M, N, K)], torch.bfloat16)]
    assert _as_key(best) in cands
    assert len(report) == len(cands) and report[0][1] is best
    assert all(report[i][0] <= report[i + 1][0] for i in range(len(report) - 1))
    again = tune.tune_gemm(A.view, B.view, reps=3)
    assert _as_key(again) == _as_key(best)
    out = sk.gemm(A.view, B.view, config=best)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    assert rel_err(as64(out), oracle(A, B, M, N, K)) <= TOL["bf16"]


def test_tune_grouped_picks_a_candidate(tmp_path, monkeypatch):
    monkeypatch.setenv("SK_TUNE_CACHE", str(tmp_path / "tune.json"))
    shapes = [(64, 1024, 2048), (300, 2048, 1024), (1000, 1024, 4096)]
    ops = []
    for i, (M, N, K) in enumerate(shapes):
        A, B = make_inputs(M, N, K, "e4m3", False, True, 70 + i, "normal")
        ops.append((A, B, torch.full((M, N), float("nan"), device=dev())))
    problems = [(A.view, B.view, out) for A, B, out in ops]
    scales = [(A.scale, B.scale) for A, B, _ in ops]
    best = tune.tune_grouped(problems, scales=scales, reps=3)
    cands = [_as_key(c) for c in tune.candidates(shapes, torch.float8_e4m3fn)]
    assert _as_key(best) in cands
    gg = sk.GroupedGemm(problems, config=best, scales=scales)
    gg.run()
    torch.cuda.synchronize()
    assert sk.check_device_error(workspace=gg.workspace) == 0
    for (A, B, out), (M, N, K) in zip(ops, shapes):
        assert rel_err(as64(out), oracle(A, B, M, N, K)) <= TOL["e4m3"]
