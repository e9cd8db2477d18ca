"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/streamk.h declares, and its host-only entry points validate
arguments and report capacity as documented."""
import ctypes
import json
import os
import re

import pytest
import torch

import paper_2407_00044_amd as sk
from paper_2407_00044_amd import _abi

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "streamk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sk_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = sk.load()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
        assert n in _abi.PROTOTYPES, f"{n} has no Python prototype"


def test_status_strings():
    for code in range(-7, 1):
        assert _abi.status_string(code)
    assert "unknown" in _abi.status_string(-99)


def _plan(M, N, K, dtype=torch.bfloat16, **kw):
    return sk.plan([(M, N, K)], dtype, sk.Config(**kw))


def _status(fn):
    with pytest.raises(_abi.StreamKError) as e:
        fn()
    return e.value.status


def test_plan_closed_forms():
    p = _plan(3840, 4096, 4096, dtype=torch.float16, tile=(256, 128), num_cu=256, mode="hybrid")
    assert (p["T"], p["S"], p["W"], p["q"], p["rho"]) == (480, 480, 30720, 120, 0)
    p = _plan(512, 512, 512, dtype=torch.float32, tile=(128, 128), mode="sk", num_cu=256,
              min_iters=1)
    assert (p["T"], p["W"], p["q"]) == (16, 256, 1)
    # fixed layout: 256-byte header, 4096 tokens, then 256 partial tiles
    assert p["workspace_bytes"] == 256 + 4 * 4096 + 256 * 128 * 128 * 4
    p = _plan(384, 384, 128, dtype=torch.float32, tile=(128, 128), mode="dp", num_cu=4)
    assert (p["T"], p["S"], p["g"], p["workspace_bytes"]) == (9, 0, 9, 0)
    p = _plan(8192, 4096, 11008, tile=(256, 128), num_cu=256)   # T mod g == 0: pure DP
    assert (p["T"], p["S"]) == (1024, 0)
    # automatic grid floor: 6 tiles x 50 iterations -> 3 pieces per tile,
    # m = 17, 17 workgroups
    p = _plan(607, 187, 3155, tile=(256, 128), num_cu=256)
    assert (p["T"], p["g"], p["q"], p["rho"]) == (6, 17, 17, 11)
    p = _plan(607, 187, 3155, tile=(256, 128), num_cu=256, min_iters=1, mode="hybrid")
    assert (p["g"], p["q"], p["rho"]) == (256, 1, 44)


def test_k_zero_keeps_one_iteration():
    p = _plan(256, 256, 0, tile=(128, 128), mode="sk", num_cu=4)
    assert p["T"] == 4 and p["W"] == 4 and p["max_iters"] == 1


def test_invalid_arguments():
    lib = sk.load()
    cfg = sk.Config(tile=(128, 128), num_cu=8).c_struct(_abi.SK_BF16)
    info = _abi.SkPlanInfo()

    def call(p, c=cfg):
        return lib.sk_plan(ctypes.byref(p), 1, ctypes.byref(c), ctypes.byref(info))

    good = _abi.SkProblem(64, 64, 64, 0, 1, 64, 64, 64, _abi.SK_BF16, 0, 1, 0, 1, 1)
    assert call(good) == _abi.SK_OK
    bad = _abi.SkProblem(*[getattr(good, f) for f, _ in _abi.SkProblem._fields_])
    bad.M = -1
    assert call(bad) == _abi.SK_ERR_INVALID_ARG
    bad.M = 64
    bad.lda = 63                                  # row-major A needs lda >= K
    assert call(bad) == _abi.SK_ERR_INVALID_ARG
    bad.lda = 64
    bad.ldc = 10
    assert call(bad) == _abi.SK_ERR_INVALID_ARG
    bad.ldc = 64
    bad.dtype_c = _abi.SK_F8E4M3                  # no e4m3 output
    assert call(bad) == _abi.SK_ERR_UNSUPPORTED
    bad.dtype_c = 0
    bad.layout_a = 7
    assert call(bad) == _abi.SK_ERR_INVALID_ARG
    bad.layout_a = 0
    # fused epilogue: activation codes 0..3, bias 4-byte aligned, reserved 0
    for act in (_abi.SK_ACT_RELU, _abi.SK_ACT_GELU, _abi.SK_ACT_SILU):
        bad.activation = act
        assert call(bad) == _abi.SK_OK
    bad.activation = 4
    assert call(bad) == _abi.SK_ERR_INVALID_ARG
    bad.activation = -1
    assert call(bad) == _abi.SK_ERR_INVALID_ARG
    bad.activation = 0
    bad.bias = 0x1002
    assert call(bad) == _abi.SK_ERR_INVALID_ARG
    bad.bias = 0x1000
    assert call(bad) == _abi.SK_OK
    bad.bias = None
    bad.reserved = 1
    assert call(bad) == _abi.SK_ERR_INVALID_ARG
    assert ctypes.sizeof(_abi.SkProblem) == 96     # the C struct's size on x86-64
    c2 = sk.Config(tile=(96, 128), num_cu=8).c_struct(_abi.SK_BF16)
    assert call(good, c2) == _abi.SK_ERR_UNSUPPORTED          # tile not built
    c3 = sk.Config(tile=(128, 128), num_cu=8).c_struct(_abi.SK_BF16)
    c3.block_k = 32
    assert call(good, c3) == _abi.SK_ERR_UNSUPPORTED          # wrong k per iteration
    c4 = sk.Config(tile=(128, 128), num_cu=8).c_struct(_abi.SK_BF16)
    c4.mode = 9
    assert call(good, c4) == _abi.SK_ERR_INVALID_ARG
    c5 = sk.Config(tile=(128, 128), num_cu=8, dp_tiles=-5).c_struct(_abi.SK_BF16)
    assert call(good, c5) == _abi.SK_ERR_INVALID_ARG


def test_schedule_capacity():
    lib = sk.load()
    p = _abi.SkProblem(384, 384, 128, 0, 0, 128, 384, 384, _abi.SK_F32, 0, 1, 0, 1, 1)
    c = sk.Config(tile=(128, 128), mode="sk", num_cu=4).c_struct(_abi.SK_F32)
    n = ctypes.c_int64()
    assert lib.sk_schedule(ctypes.byref(p), 1, ctypes.byref(c), None, 0, ctypes.byref(n)) == 0
    assert n.value == 12
    segs = (_abi.SkSegment * 5)()
    assert lib.sk_schedule(ctypes.byref(p), 1, ctypes.byref(c), segs, 5,
                           ctypes.byref(n)) == _abi.SK_ERR_CAPACITY


def test_tile_menu():
    assert sk.supported_tiles(torch.float32) == [(128, 128, 32)]
    for dt in (torch.float16, torch.bfloat16):
        assert sk.supported_tiles(dt) == [(128, 128, 64), (256, 128, 64), (256, 256, 64)]
    assert (64, 128, 128) in sk.supported_tiles(torch.float8_e4m3fn)


def test_operand_layout_inference():
    from paper_2407_00044_amd.api import operand_layout
    x = torch.zeros(6, 10)
    assert operand_layout(x) == (0, 10)
    assert operand_layout(x.t()) == (1, 10)
    assert operand_layout(torch.zeros(6, 16)[:, :10]) == (0, 16)
    with pytest.raises(ValueError):
        operand_layout(torch.zeros(6, 10)[:, ::2])


def test_workspace_init_rejects_bad_args():
    lib = sk.load()
    assert lib.sk_workspace_init(None, 64, None) == _abi.SK_ERR_INVALID_ARG
    assert lib.sk_workspace_init(None, 0, None) == _abi.SK_OK


def test_tuner_candidates():
    from paper_2407_00044_amd import tune
    c = tune.candidates([(3840, 4096, 4096)], torch.bfloat16, num_cu=256)
    modes = {(x.tile, x.mode, x.dp_tiles) for x in c}
    assert ((256, 128), "hybrid", -1) in modes and ((256, 256), "dp", -1) in modes
    assert ((256, 256), "auto", -1) in modes
    assert ((128, 128), "sk", -1) in modes
    # T = 480 tiles of 256x128 on 256 workgroups: one-tile remainder keeps 256 DP tiles
    assert ((256, 128), "hybrid", 256) in modes


def test_tuner_cache_round_trip_keeps_every_schedule_field():
    from paper_2407_00044_amd import tune
    c = sk.Config(tile=(256, 128), mode="hybrid", num_cu=200, dp_tiles=128, group_m=0,
                  min_iters=1)
    d = json.loads(json.dumps(tune.config_to_dict(c)))
    assert tune.config_from_dict(d) == c


def test_default_tile_rule():
    bf = torch.bfloat16
    assert sk.default_tile(3840, 4096, 4096, bf) == (256, 256)       # 240 tiles >= 0.55/CU
    assert sk.default_tile(4826, 1341, 13813, bf) == (256, 256)     # 114 tiles x 216 iterations
    assert sk.default_tile(5222, 1459, 1260, bf) == (256, 128)      # 252 tiles >= 0.9/CU
    assert sk.default_tile(2048, 2048, 4096, bf) == (128, 128)
    assert sk.default_tile(512, 512, 512, torch.float32) == (128, 128)
    assert sk.default_tile(48, 1024, 2048, torch.float8_e4m3fn) == (64, 128)
    e4 = torch.float8_e4m3fn
    assert sk.default_tile(4826, 1341, 13813, e4) == (256, 128)    # 209 tiles x 108 iterations
    assert sk.default_tile(2073, 2069, 1620, e4) == (128, 128)     # 153 tiles x 13 iterations
    assert sk.default_tile(3840, 4096, 4096, e4) == (256, 128)


def test_tuner_cache_unwritable_location_is_harmless(monkeypatch, tmp_path):
    from paper_2407_00044_amd import tune
    blocker = tmp_path / "file"
    blocker.write_text("x")
    monkeypatch.setenv("SK_TUNE_CACHE", str(blocker / "sub" / "tune.json"))
    tune._store_cache({"k": 1})                 # parent is a file: cannot be created
    assert tune._load_cache() == {}


def test_tile_span_limit_and_large_problems():
    # buffer offsets are 32-bit relative to a tile's first element: a tile
    # whose furthest element lies 2^31 bytes or more away is rejected
    lib = sk.load()
    cfg = sk.Config(tile=(128, 128), num_cu=256).c_struct(_abi.SK_BF16)
    info = _abi.SkPlanInfo()
    K = 64
    near = (2 ** 31 // 2 - K) // 127                 # 127 * lda + K elements just fit
    p = _abi.SkProblem(4096, 4096, K, 0, 1, near, K, 4096, _abi.SK_BF16, 0, 1, 0, 1, 1)
    assert lib.sk_plan(ctypes.byref(p), 1, ctypes.byref(cfg), ctypes.byref(info)) == _abi.SK_OK
    p.lda = near + 1
    assert lib.sk_plan(ctypes.byref(p), 1, ctypes.byref(cfg), ctypes.byref(info)) == \
        _abi.SK_ERR_UNSUPPORTED
    # a large problem: 65536^3 on 128x128 tiles, 256 workgroups
    big = _abi.SkProblem(65536, 65536, 65536, 0, 1, 65536, 65536, 65536, _abi.SK_BF16, 0,
                         1, 0, 1, 1)
    hyb = sk.Config(tile=(128, 128), num_cu=256, mode="hybrid").c_struct(_abi.SK_BF16)
    assert lib.sk_plan(ctypes.byref(big), 1, ctypes.byref(hyb), ctypes.byref(info)) == _abi.SK_OK
    assert info.T == 512 * 512 and info.S == 0        # T mod g == 0: pure data-parallel


def test_mx_entry_point_host_checks():
    # host-side rejections of sk_gemm_mx (nothing is launched, no GPU touched)
    lib = _abi.load()
    cfg = sk.Config(tile=(128, 128), num_cu=8).c_struct(_abi.SK_MXF8E4M3)

    def prob(M, N, K, la=_abi.SK_ROW_MAJOR, lb=_abi.SK_COL_MAJOR, dt=_abi.SK_MXF8E4M3):
        lda = K if la == _abi.SK_ROW_MAJOR else M
        ldb = K if lb == _abi.SK_COL_MAJOR else N
        return _abi.SkProblem(M, N, K, la, lb, lda, ldb, N, dt, _abi.SK_F32, 1.0, 0.0, 1.0, 1.0)

    fake = ctypes.c_void_p(1 << 20)          # 16-byte aligned, never dereferenced

    def call(p, lds=8, sa=fake, sb=fake, a=fake):
        return lib.sk_gemm_mx(ctypes.byref(p), a, fake, sa, lds, sb, lds, None, fake, None, 0,
                              ctypes.byref(cfg), None)
    # K not a multiple of 128, or M/N-contiguous operands: not built
    assert call(prob(256, 256, 192)) == _abi.SK_ERR_UNSUPPORTED
    assert call(prob(256, 256, 256, la=_abi.SK_COL_MAJOR)) == _abi.SK_ERR_UNSUPPORTED
    assert call(prob(256, 256, 256, lb=_abi.SK_ROW_MAJOR)) == _abi.SK_ERR_UNSUPPORTED
    # A not 16-byte aligned: unsupported; scale pitch too short or unaligned
    assert call(prob(256, 256, 256), a=ctypes.c_void_p((1 << 20) + 4)) == _abi.SK_ERR_UNSUPPORTED
    assert call(prob(256, 256, 256), lds=4) == _abi.SK_ERR_INVALID_ARG
    assert call(prob(256, 256, 256), lds=10) == _abi.SK_ERR_INVALID_ARG
    assert call(prob(256, 256, 256), sa=None) == _abi.SK_ERR_INVALID_ARG
    assert call(prob(256, 256, 256), sb=ctypes.c_void_p((1 << 20) + 2)) == _abi.SK_ERR_INVALID_ARG
    # MXFP8 needs its scales: plain sk_gemm refuses it, and sk_gemm_mx
    # refuses any other input type
    p = prob(256, 256, 256)
    assert lib.sk_gemm(ctypes.byref(p), fake, fake, None, fake, None, 0, ctypes.byref(cfg),
                       None) == _abi.SK_ERR_INVALID_ARG
    cfg8 = sk.Config(tile=(128, 128), num_cu=8).c_struct(_abi.SK_F8E4M3)
    p8 = prob(256, 256, 256, dt=_abi.SK_F8E4M3)
    assert lib.sk_gemm_mx(ctypes.byref(p8), fake, fake, fake, 8, fake, 8, None, fake, None, 0,
                          ctypes.byref(cfg8), None) == _abi.SK_ERR_INVALID_ARG
    # the tile menu: 256x128 and 128x128
    assert sk.supported_tiles(_abi.SK_MXF8E4M3) == [(128, 128, 128), (256, 128, 128)]


def test_grouped_mx_host_checks():
    # host-side rejections of sk_grouped_prepare(_mx) for MXFP8 problems; each
    # is raised before the descriptors would be copied (no GPU touched)
    lib = _abi.load()
    cfg = sk.Config(tile=(128, 128), num_cu=8).c_struct(_abi.SK_MXF8E4M3)
    n = 2
    probs = (_abi.SkProblem * n)()
    for i, (M, N, K) in enumerate([(256, 256, 256), (100, 300, 512)]):
        probs[i] = _abi.SkProblem(M, N, K, _abi.SK_ROW_MAJOR, _abi.SK_COL_MAJOR, K, K, N,
                                  _abi.SK_MXF8E4M3, _abi.SK_F32, 1.0, 0.0, 1.0, 1.0)
    fake = 1 << 20
    ptr = lambda v: (ctypes.c_void_p * n)(*([v] * n))          # noqa: E731
    lds = lambda v: (ctypes.c_int64 * n)(*([v] * n))           # noqa: E731
    plan = _abi.SkGroupedPlan()
    desc = ctypes.c_void_p(fake)
    dbytes = 1 << 16
    # plain prepare: MXFP8 problems need their scales
    assert lib.sk_grouped_prepare(probs, ptr(fake), ptr(fake), None, ptr(fake), n,
                                  ctypes.byref(cfg), desc, dbytes, ctypes.byref(plan),
                                  None) == _abi.SK_ERR_INVALID_ARG

    def call(sa=fake, sb=fake, la=16, lb=16):
        return lib.sk_grouped_prepare_mx(probs, ptr(fake), ptr(fake), ptr(sa), lds(la), ptr(sb),
                                         lds(lb), None, ptr(fake), n, ctypes.byref(cfg), desc,
                                         dbytes, ctypes.byref(plan), None)
    assert call(sa=fake + 2) == _abi.SK_ERR_INVALID_ARG          # scale rows 4-byte aligned
    assert call(lb=6) == _abi.SK_ERR_INVALID_ARG                 # pitch a multiple of 4
    assert call(la=8) == _abi.SK_ERR_INVALID_ARG                 # >= K/32 = 16 bytes
    assert lib.sk_grouped_prepare_mx(probs, ptr(fake), ptr(fake), None, lds(16), ptr(fake),
                                     lds(16), None, ptr(fake), n, ctypes.byref(cfg), desc,
                                     dbytes, ctypes.byref(plan), None) == _abi.SK_ERR_INVALID_ARG
    # K not a multiple of 128 in one problem: not built
    probs[1].K = 320
    probs[1].lda = probs[1].ldb = 320
    assert call() == _abi.SK_ERR_UNSUPPORTED
    # the MXFP8 prepare refuses other input types
    cfg8 = sk.Config(tile=(128, 128), num_cu=8).c_struct(_abi.SK_F8E4M3)
    for i in range(n):
        probs[i].dtype_ab = _abi.SK_F8E4M3
        probs[i].K = probs[i].lda = probs[i].ldb = 256
    assert lib.sk_grouped_prepare_mx(probs, ptr(fake), ptr(fake), ptr(fake), lds(16), ptr(fake),
                                     lds(16), None, ptr(fake), n, ctypes.byref(cfg8), desc,
                                     dbytes, ctypes.byref(plan), None) == _abi.SK_ERR_INVALID_ARG


def test_mx4_entry_point_host_checks():
    # MXFP4 through sk_gemm_mx: whole 256-element iterations and rows of a
    # multiple of 16 bytes (32 elements), else unsupported (nothing launched)
    lib = _abi.load()
    cfg = sk.Config(tile=(128, 128), num_cu=8).c_struct(_abi.SK_MXF4E2M1)
    assert cfg.block_k == 256
    fake = ctypes.c_void_p(1 << 20)

    def call(M, N, K, lda=None, ldb=None, lds=16):
        p = _abi.SkProblem(M, N, K, _abi.SK_ROW_MAJOR, _abi.SK_COL_MAJOR, lda or K, ldb or K, N,
                           _abi.SK_MXF4E2M1, _abi.SK_F32, 1.0, 0.0, 1.0, 1.0)
        return lib.sk_gemm_mx(ctypes.byref(p), fake, fake, fake, lds, fake, lds, None, fake,
                              None, 0, ctypes.byref(cfg), None)
    assert call(256, 256, 384) == _abi.SK_ERR_UNSUPPORTED          # K % 256
    assert call(256, 256, 512, lda=528) == _abi.SK_ERR_UNSUPPORTED   # 264-byte rows
    assert call(256, 256, 512, ldb=520) == _abi.SK_ERR_UNSUPPORTED
    assert call(256, 256, 512, lds=8) == _abi.SK_ERR_INVALID_ARG     # < K/32 scale bytes
    assert sk.supported_tiles(_abi.SK_MXF4E2M1) == [(128, 128, 256), (256, 128, 256)]
    # the planner counts K in elements: 512 / 256 = 2 iterations per tile
    p = _abi.SkProblem(256, 256, 512, _abi.SK_ROW_MAJOR, _abi.SK_COL_MAJOR, 512, 512, 256,
                       _abi.SK_MXF4E2M1, _abi.SK_F32, 1.0, 0.0, 1.0, 1.0)
    info = _abi.SkPlanInfo()
    assert lib.sk_plan(ctypes.byref(p), 1, ctypes.byref(cfg), ctypes.byref(info)) == 0
    assert info.T == 4 and info.max_iters == 2


def test_transpose_rejects_bad_arguments_on_the_host():
    # every check runs before anything is enqueued (no GPU needed)
    lib = sk.load()
    c = ctypes.c_void_p
    buf_a, buf_b = c(0x100000), c(0x900000)
    bad = [
        (buf_a, 4, 5, 5, buf_b, 4, 3),        # 3-byte elements
        (buf_a, -1, 5, 5, buf_b, 4, 2),       # negative rows
        (buf_a, 4, 5, 4, buf_b, 4, 2),        # ld_in < cols
        (buf_a, 4, 5, 5, buf_b, 3, 2),        # ld_out < rows
        (c(None), 4, 5, 5, buf_b, 4, 2),      # null input
        (buf_a, 4, 5, 5, c(None), 4, 2),      # null output
        (buf_a, 4, 5, 5, c(0x100000 + 8), 4, 2),   # overlapping matrices
    ]
    for args in bad:
        assert lib.sk_transpose(*args, c(None)) == _abi.SK_ERR_INVALID_ARG, args
    # empty matrices: nothing to do, no pointers needed
    assert lib.sk_transpose(c(None), 0, 5, 5, c(None), 1, 2, c(None)) == _abi.SK_OK
    assert lib.sk_transpose(c(None), 7, 0, 1, c(None), 7, 4, c(None)) == _abi.SK_OK


def test_pack_rule():
    # the BF16 linear layer's backward products pack, and so do products
    # with a short M or N but long K; short K, small products, small e4m3
    # products and FP32 do not
    assert sk.pack_pays(8192, 4096, 11008, torch.bfloat16)
    assert sk.pack_pays(11008, 4096, 8192, torch.bfloat16)
    assert sk.pack_pays(1024, 4096, 4096, torch.bfloat16)
    assert sk.pack_pays(4096, 4096, 4096, torch.float8_e4m3fn)
    assert not sk.pack_pays(4096, 4096, 1024, torch.bfloat16)
    assert not sk.pack_pays(1024, 1024, 4096, torch.bfloat16)
    assert not sk.pack_pays(2048, 2048, 2048, torch.float8_e4m3fn)
    assert not sk.pack_pays(8192, 4096, 11008, torch.float32)
    assert not sk.pack_pays(320, 384, 448, torch.float16)


def test_mx6_entry_point_host_checks():
    # MXFP6 through sk_gemm_mx: whole 128-element iterations and rows of a
    # multiple of 64 elements (48 bytes, a multiple of 16); nothing launched
    lib = _abi.load()
    fake = ctypes.c_void_p(1 << 20)
    for dt in (_abi.SK_MXF6E2M3, _abi.SK_MXF6E3M2):
        cfg = sk.Config(tile=(128, 128), num_cu=8).c_struct(dt)
        assert cfg.block_k == 128

        def call(M, N, K, lda, ldb, lds=8):
            p = _abi.SkProblem(M, N, K, _abi.SK_ROW_MAJOR, _abi.SK_COL_MAJOR, lda, ldb, N, dt,
                               _abi.SK_F32, 1.0, 0.0, 1.0, 1.0)
            return lib.sk_gemm_mx(ctypes.byref(p), fake, fake, fake, lds, fake, lds, None, fake,
                                  None, 0, ctypes.byref(cfg), None)
        assert call(256, 256, 192, 192, 192) == _abi.SK_ERR_UNSUPPORTED    # K % 128
        assert call(256, 256, 256, 288, 256) == _abi.SK_ERR_UNSUPPORTED    # lda % 64
        assert call(256, 256, 256, 256, 320, lds=4) == _abi.SK_ERR_INVALID_ARG   # scales < K/32
        # plain sk_gemm refuses an MX type
        p = _abi.SkProblem(256, 256, 256, _abi.SK_ROW_MAJOR, _abi.SK_COL_MAJOR, 256, 256, 256,
                           dt, _abi.SK_F32, 1.0, 0.0, 1.0, 1.0)
        assert lib.sk_gemm(ctypes.byref(p), fake, fake, None, fake, None, 0, ctypes.byref(cfg),
                           None) == _abi.SK_ERR_INVALID_ARG


def test_mx8_e5m2_entry_point_host_checks():
    # MXFP8 with e5m2 elements takes the e4m3 rules; a type past the last
    # one is refused; the binding refuses mixed element formats
    lib = _abi.load()
    fake = ctypes.c_void_p(1 << 20)
    dt = _abi.SK_MXF8E5M2
    cfg = sk.Config(tile=(128, 128), num_cu=8).c_struct(dt)
    assert cfg.block_k == 128

    def call(M, N, K, la=_abi.SK_ROW_MAJOR, dtype=dt, lds=8):
        p = _abi.SkProblem(M, N, K, la, _abi.SK_COL_MAJOR, K if la == _abi.SK_ROW_MAJOR else M,
                           K, N, dtype, _abi.SK_F32, 1.0, 0.0, 1.0, 1.0)
        return lib.sk_gemm_mx(ctypes.byref(p), fake, fake, fake, lds, fake, lds, None, fake,
                              None, 0, ctypes.byref(cfg), None)
    assert call(256, 256, 192) == _abi.SK_ERR_UNSUPPORTED                  # K % 128
    assert call(256, 256, 256, la=_abi.SK_COL_MAJOR) == _abi.SK_ERR_UNSUPPORTED
    assert call(256, 256, 256, lds=4) == _abi.SK_ERR_INVALID_ARG          # scales < K/32
    # the per-tensor type takes no block scales; a type past the last is unknown
    assert call(256, 256, 256, dtype=_abi.SK_F8E5M2) == _abi.SK_ERR_INVALID_ARG
    assert call(256, 256, 256, dtype=_abi.SK_F8E5M2 + 1) == _abi.SK_ERR_UNSUPPORTED
    a = torch.zeros((64, 128), dtype=torch.float8_e4m3fn)
    b = torch.zeros((128, 64), dtype=torch.float8_e5m2)
    s = torch.zeros((64, 8), dtype=torch.uint8)
    with pytest.raises(TypeError):
        sk.gemm_mx(a, b, s, s)


def test_f8_e5m2_plans_as_e4m3():
    # per-tensor e5m2 takes e4m3's iteration depth, tile menu and schedule
    cfg = sk.Config(tile=(64, 128), mode="hybrid", num_cu=64, min_iters=1)
    for shape in [(700, 520, 1000), (64, 4096, 8192)]:
        assert sk.plan([shape], torch.float8_e5m2, cfg) == \
            sk.plan([shape], torch.float8_e4m3fn, cfg)
    assert sk.default_tile(64, 4096, 4096, torch.float8_e5m2) == (64, 128)
    assert sk.pack_pays(4096, 4096, 4096, torch.float8_e5m2) == \
        sk.pack_pays(4096, 4096, 4096, torch.float8_e4m3fn)
