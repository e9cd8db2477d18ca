"""Torch-facing API of the Stream-K GEMM (argument marshalling only).

Torch supplies device memory and streams; every arithmetic step of a GEMM
runs in libstreamk.so's HIP kernels.  Functions here infer layouts from
tensor strides, fill the C structures, manage the reusable workspace and
translate status codes into exceptions.
"""
import ctypes
from dataclasses import dataclass, replace

import torch

from . import _abi
from ._abi import (SK_COL_MAJOR, SK_ROW_MAJOR, SkConfig, SkDebug, SkGroupedPlan,
                   SkPlanInfo, SkProblem, SkSegment, check, load)

DTYPE_CODES = {torch.float32: _abi.SK_F32, torch.float16: _abi.SK_F16,
               torch.bfloat16: _abi.SK_BF16, torch.float8_e4m3fn: _abi.SK_F8E4M3,
               torch.float8_e5m2: _abi.SK_F8E5M2}
OUT_CODES = {torch.float32: _abi.SK_F32, torch.float16: _abi.SK_F16,
             torch.bfloat16: _abi.SK_BF16}
K_PER_ITER = {_abi.SK_F32: 32, _abi.SK_F16: 64, _abi.SK_BF16: 64, _abi.SK_F8E4M3: 128,
              _abi.SK_MXF8E4M3: 128, _abi.SK_MXF4E2M1: 256, _abi.SK_MXF6E2M3: 128,
              _abi.SK_MXF6E3M2: 128, _abi.SK_MXF8E5M2: 128,
              _abi.SK_F8E5M2: 128}
# MXFP8 element formats: torch code dtype -> sk_dtype
MX8_CODES = {torch.float8_e4m3fn: _abi.SK_MXF8E4M3, torch.float8_e5m2: _abi.SK_MXF8E5M2}

SEGMENT_FIELDS = ("wg", "problem", "tile", "tile_m", "tile_n", "k_begin", "k_end",
                  "role", "npeers")


@dataclass(frozen=True)
class Config:
    """Launch configuration (mirrors sk_config).

    tile: (block_m, block_n); block_k follows from the input type.
    mode: 'auto' (hybrid that splits tiles only where the cost model says
    Stream-K beats data-parallel waves), 'hybrid' (data-parallel + Stream-K,
    two-tile rule), 'sk' or 'dp' (baseline grid).
    num_cu: compute units (0 = all); wg_per_cu: persistent workgroups per CU.
    dp_tiles: -1 = two-tile hybrid rule, else number of data-parallel tiles.
    group_m: tile order (0 row-major, > 0 bands of group_m rows, -1 automatic).
    min_iters: Stream-K grid floor (0 = automatic, 1 = always g workgroups).
    """
    tile: tuple = (256, 128)
    mode: str = "auto"
    num_cu: int = 0
    wg_per_cu: int = 1
    dp_tiles: int = -1
    group_m: int = -1
    xcd_remap: int = 1
    spin_limit: int = 0
    min_iters: int = 0

    def c_struct(self, dtype_code):
        return SkConfig(self.tile[0], self.tile[1], K_PER_ITER[dtype_code], self.num_cu,
                        self.wg_per_cu, _abi.MODES[self.mode], self.dp_tiles, self.group_m,
                        self.xcd_remap, self.spin_limit, self.min_iters)


def default_tile(M, N, K, dtype, cus=256):
    """Tile for a problem when none is given.

    Larger tiles need fewer operand bytes per flop but leave more compute
    units idle or split more.  Measured on the BF16 shape sweep (auto mode):
    256x256 (f16/bf16, any layout) pays once it yields ~0.55 tiles per CU, or
    once its MAC iterations reach 32 per CU, where Stream-K spreads a few
    long-K tiles over every CU; 256x128 pays from ~0.9 tiles per CU; 128x128
    is best below.  e4m3 (measured on the same shapes in e4m3): no 256x256
    (it lost on most shapes), and 256x128 also once its MAC iterations reach
    32 per CU."""
    code = DTYPE_CODES[dtype]
    if code == _abi.SK_F32:
        return (128, 128)
    if code in (_abi.SK_F8E4M3, _abi.SK_F8E5M2) and M <= 64:
        return (64, 128)
    iters = max(1, -(-K // K_PER_ITER[code]))
    t256 = -(-M // 256) * -(-N // 256)
    if code in (_abi.SK_F16, _abi.SK_BF16) and M >= 256 and N >= 256 and \
            (t256 * 100 >= cus * 55 or t256 * iters >= 32 * cus):
        return (256, 256)
    t256x128 = -(-M // 256) * -(-N // 128)
    if M >= 256 and t256x128 * 10 >= cus * 9:
        return (256, 128)
    if code in (_abi.SK_F8E4M3, _abi.SK_F8E5M2) and M >= 256 and t256x128 * iters >= 32 * cus:
        return (256, 128)
    return (128, 128)


def operand_layout(t, prefer=None):
    """(layout, ld) of a 2-D tensor with unit stride in one dimension.

    An empty matrix has no layout of its own: with `prefer` given it takes
    that layout (with the smallest valid leading dimension)."""
    if t.dim() != 2:
        raise ValueError("operands must be 2-D")
    r, c = t.shape
    if t.numel() == 0 and prefer is not None:
        return prefer, max(1, c if prefer == SK_ROW_MAJOR else r)
    s0, s1 = t.stride()
    if (s1 == 1 or c <= 1) and s0 >= max(1, c):
        return SK_ROW_MAJOR, max(s0, 1)
    if (s0 == 1 or r <= 1) and s1 >= max(1, r):
        return SK_COL_MAJOR, max(s1, 1)
    raise ValueError(f"operand with strides {t.stride()} is neither row- nor column-major")


def _problem(A, B, C, alpha, beta, scale_a, scale_b, prefer=(None, None)):
    M, K = A.shape
    K2, N = B.shape
    if K != K2 or tuple(C.shape) != (M, N):
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, "
                         f"C {tuple(C.shape)}")
    if A.dtype != B.dtype or A.dtype not in DTYPE_CODES:
        raise TypeError(f"A and B must share one of {list(DTYPE_CODES)}")
    if C.dtype not in OUT_CODES:
        raise TypeError(f"C must be one of {list(OUT_CODES)}")
    la, lda = operand_layout(A, prefer[0])
    lb, ldb = operand_layout(B, prefer[1])
    if C.stride(1) != 1 and N > 1:
        raise ValueError("C must be row-major")
    ldc = max(C.stride(0), N, 1)
    return SkProblem(M, N, K, la, lb, lda, ldb, ldc, DTYPE_CODES[A.dtype],
                     OUT_CODES[C.dtype], alpha, beta, scale_a, scale_b)


ACTIVATIONS = {"none": _abi.SK_ACT_NONE, "relu": _abi.SK_ACT_RELU,
               "gelu": _abi.SK_ACT_GELU, "silu": _abi.SK_ACT_SILU}


def _set_epilogue(p, bias, activation, device):
    """Fused epilogue fields of a problem: bias (N FP32 values on the GPU,
    or None) added to every row, then the activation (see ACTIVATIONS)."""
    if activation not in ACTIVATIONS:
        raise ValueError(f"activation must be one of {list(ACTIVATIONS)}")
    p.activation = ACTIVATIONS[activation]
    if bias is not None:
        if (bias.dtype != torch.float32 or bias.dim() != 1 or bias.numel() != p.N
                or bias.stride(0) != 1 or bias.device != device):
            raise ValueError("bias: contiguous float32 vector of N values on the GPU")
        p.bias = bias.data_ptr()
    return p


class Workspace:
    """Reusable fixup workspace for one device and stream (grows on demand;
    zeroed with the library's fill kernel whenever it is (re)allocated)."""

    def __init__(self, device=None):
        self.device = torch.device(device or "cuda")
        self.buf = None

    def get(self, nbytes, stream):
        if nbytes == 0:
            return None, 0
        if self.buf is None or self.buf.numel() < nbytes:
            size = max(nbytes, 1 << 20)
            self.buf = torch.empty(size, dtype=torch.uint8, device=self.device)
            check("sk_workspace_init",
                  load().sk_workspace_init(ctypes.c_void_p(self.buf.data_ptr()),
                                           self.buf.numel(), ctypes.c_void_p(stream)))
        return self.buf.data_ptr(), self.buf.numel()


_workspaces = {}


def workspace_for(device, stream):
    key = (torch.device(device).index, stream)
    ws = _workspaces.get(key)
    if ws is None:
        ws = _workspaces[key] = Workspace(device)
    return ws


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def gemm(A, B, C=None, *, alpha=1.0, beta=0.0, out=None, out_dtype=torch.float32,
         scale_a=1.0, scale_b=1.0, bias=None, activation="none", config=None,
         workspace=None, stream=None, pack=False):
    """out = act(alpha * scale_a * scale_b * (A @ B) + beta * C + bias) on the
    GPU (bias and act optional: the fused epilogue; see ACTIVATIONS).

    A (M x K) and B (K x N) may each be row- or column-major (unit stride in
    one dimension); out and C are row-major.  With C given and out None the
    update is in place (out = C).  pack (False, True or "auto": where
    pack_pays) first copies M- or N-major operands K-contiguous
    (sk_transpose, on the same stream); the result is the same bit for bit."""
    lib = load()
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("operands must be on the GPU")
    if pack not in (True, False, "auto"):
        raise ValueError('pack must be True, False or "auto"')
    M, N = A.shape[0], B.shape[1]
    if pack is True or (pack == "auto" and A.dtype in DTYPE_CODES and
                        pack_pays(M, N, A.shape[1], A.dtype)):
        A, B = k_contiguous(A, "a", stream), k_contiguous(B, "b", stream)
    if out is None:
        out = C if (C is not None and beta != 0.0) else torch.empty(
            (M, N), dtype=out_dtype, device=A.device)
    if beta != 0.0 and C is None:
        raise ValueError("beta != 0 needs C")
    p = _set_epilogue(_problem(A, B, out, alpha, beta, scale_a, scale_b), bias, activation,
                      A.device)
    cfg = config or Config(tile=default_tile(M, N, A.shape[1], A.dtype))
    if C is not None and beta != 0.0:
        if tuple(C.shape) != (M, N) or C.dtype != out.dtype or C.stride() != out.stride():
            raise ValueError("C must match out in shape, dtype and strides")
    c = cfg.c_struct(p.dtype_ab)
    sp = _stream_ptr(stream)
    nbytes = ctypes.c_size_t()
    check("sk_workspace_size", lib.sk_workspace_size(ctypes.byref(p), 1, ctypes.byref(c),
                                                      ctypes.byref(nbytes)))
    ws = workspace or workspace_for(A.device, sp)
    wptr, wlen = ws.get(nbytes.value, sp)
    cin = C.data_ptr() if (C is not None and beta != 0.0) else None
    check("sk_gemm", lib.sk_gemm(ctypes.byref(p), ctypes.c_void_p(A.data_ptr()),
                                 ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(cin),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(wptr),
                                 wlen, ctypes.byref(c), ctypes.c_void_p(sp)))
    return out


def gemm_mx(A, B, scale_a, scale_b, C=None, *, alpha=1.0, beta=0.0, out=None,
            out_dtype=torch.float32, bias=None, activation="none", config=None,
            workspace=None, stream=None):
    """MXFP8 GEMM through sk_gemm_mx: A (M x K, row-major) and B (K x N,
    column-major) hold e4m3 or e5m2 codes (torch.float8_e4m3fn or
    torch.float8_e5m2, both operands alike); scale_a (M x >= K/32)
    and scale_b (N x >= K/32) hold one E8M0 byte (uint8, 2^(e-127)) per 32
    K-values of each row of A and column of B, rows contiguous.
    out = act(alpha * sum_k (A * 2^(sa-127)) (B * 2^(sb-127)) + beta * C + bias)."""
    lib = load()
    if A.dtype not in MX8_CODES or B.dtype != A.dtype:
        raise TypeError("MXFP8 operands: torch.float8_e4m3fn or torch.float8_e5m2 codes, "
                        "both alike")
    dt = MX8_CODES[A.dtype]
    for s_ in (scale_a, scale_b):
        if s_.dtype != torch.uint8 or s_.dim() != 2 or s_.stride(1) != 1 or not s_.is_cuda:
            raise TypeError("block scales: 2-D uint8 GPU tensors with contiguous rows")
    M, N = A.shape[0], B.shape[1]
    if out is None:
        out = C if (C is not None and beta != 0.0) else torch.empty(
            (M, N), dtype=out_dtype, device=A.device)
    if beta != 0.0 and C is None:
        raise ValueError("beta != 0 needs C")
    # the descriptor takes its layout from byte views of the codes
    p = _set_epilogue(_problem(A.view(torch.float8_e4m3fn), B.view(torch.float8_e4m3fn), out,
                               alpha, beta, 1.0, 1.0), bias, activation, A.device)
    p.dtype_ab = dt
    if scale_a.shape[0] != M or scale_b.shape[0] != N:
        raise ValueError("one scale row per row of A and per column of B")
    if config is None:
        tile = default_tile(M, N, A.shape[1], torch.float8_e4m3fn)
        config = Config(tile=tile if tile in ((256, 128), (128, 128)) else (128, 128))
    cfg = config
    c = cfg.c_struct(dt)
    sp = _stream_ptr(stream)
    nbytes = ctypes.c_size_t()
    check("sk_workspace_size", lib.sk_workspace_size(ctypes.byref(p), 1, ctypes.byref(c),
                                                      ctypes.byref(nbytes)))
    ws = workspace or workspace_for(A.device, sp)
    wptr, wlen = ws.get(nbytes.value, sp)
    cin = C.data_ptr() if (C is not None and beta != 0.0) else None
    check("sk_gemm_mx", lib.sk_gemm_mx(
        ctypes.byref(p), ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
        ctypes.c_void_p(scale_a.data_ptr()), max(1, scale_a.stride(0)),
        ctypes.c_void_p(scale_b.data_ptr()), max(1, scale_b.stride(0)), ctypes.c_void_p(cin),
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(wptr), wlen, ctypes.byref(c),
        ctypes.c_void_p(sp)))
    return out


def _fp4_bytes(t):
    """Packed MXFP4 operand (torch.float4_e2m1fn_x2 or uint8, two elements
    per byte) as uint8."""
    if t.dtype == torch.float4_e2m1fn_x2:
        return t.view(torch.uint8)
    if t.dtype != torch.uint8:
        raise TypeError("MXFP4 operands: packed bytes (uint8 or torch.float4_e2m1fn_x2)")
    return t


def _mx4_problem(A, B, out, alpha, beta):
    """sk_problem of an MXFP4 product: A (M x K/2 bytes, row-major), B (K/2 x
    N bytes, column-major), out row-major M x N; sizes in elements."""
    A, B = _fp4_bytes(A), _fp4_bytes(B)
    if (A.numel() and A.stride(1) != 1) or (B.numel() and B.stride(0) != 1):
        raise ValueError("MXFP4: A row-major and B column-major")
    M, K, N = A.shape[0], 2 * A.shape[1], B.shape[1]
    if B.shape[0] * 2 != K or tuple(out.shape) != (M, N):
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)} (bytes), "
                         f"out {tuple(out.shape)}")
    if out.dtype not in OUT_CODES or (out.stride(1) != 1 and N > 1):
        raise ValueError("out must be a row-major float32/float16/bfloat16 tensor")
    return SkProblem(M, N, K, SK_ROW_MAJOR, SK_COL_MAJOR, max(2 * A.stride(0), K, 1),
                     max(2 * B.stride(1), K, 1), max(out.stride(0), N, 1), _abi.SK_MXF4E2M1,
                     OUT_CODES[out.dtype], alpha, beta, 1.0, 1.0)


def gemm_mx4(A, B, scale_a, scale_b, C=None, *, alpha=1.0, beta=0.0, out=None,
             out_dtype=torch.float32, bias=None, activation="none", config=None,
             workspace=None, stream=None):
    """MXFP4 GEMM through sk_gemm_mx: A (M x K/2 bytes, row-major) and B
    (K/2 x N bytes, column-major: the transpose of an N x K/2 row-major
    array) hold E2M1 codes two per byte, element 2j in the low nibble of
    byte j; scale_a (M x >= K/32) and scale_b (N x >= K/32) hold one E8M0
    byte per 32 K-values, rows contiguous.
    out = act(alpha * sum_k (A * 2^(sa-127)) (B * 2^(sb-127)) + beta * C + bias)."""
    lib = load()
    A, B = _fp4_bytes(A), _fp4_bytes(B)
    for s_ in (scale_a, scale_b):
        if s_.dtype != torch.uint8 or s_.dim() != 2 or s_.stride(1) != 1 or not s_.is_cuda:
            raise TypeError("block scales: 2-D uint8 GPU tensors with contiguous rows")
    if not (A.is_cuda and B.is_cuda) or A.stride(1) != 1 or B.stride(0) != 1:
        raise ValueError("A row-major and B column-major on the GPU")
    M, K, N = A.shape[0], 2 * A.shape[1], B.shape[1]
    if B.shape[0] * 2 != K:
        raise ValueError("A and B disagree on K")
    if out is None:
        out = C if (C is not None and beta != 0.0) else torch.empty(
            (M, N), dtype=out_dtype, device=A.device)
    if beta != 0.0 and C is None:
        raise ValueError("beta != 0 needs C")
    if scale_a.shape[0] != M or scale_b.shape[0] != N:
        raise ValueError("one scale row per row of A and per column of B")
    p = _set_epilogue(_mx4_problem(A, B, out, alpha, beta), bias, activation, A.device)
    if config is None:
        # the bf16 rule (the same four 16-byte steps per iteration) on the
        # MXFP4 menu: 256x128 and 128x128
        tile = default_tile(M, N, K, torch.bfloat16)
        config = Config(tile=(256, 128) if tile[0] == 256 else (128, 128))
    c = config.c_struct(_abi.SK_MXF4E2M1)
    sp = _stream_ptr(stream)
    nbytes = ctypes.c_size_t()
    check("sk_workspace_size", lib.sk_workspace_size(ctypes.byref(p), 1, ctypes.byref(c),
                                                      ctypes.byref(nbytes)))
    ws = workspace or workspace_for(A.device, sp)
    wptr, wlen = ws.get(nbytes.value, sp)
    cin = C.data_ptr() if (C is not None and beta != 0.0) else None
    check("sk_gemm_mx", lib.sk_gemm_mx(
        ctypes.byref(p), ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
        ctypes.c_void_p(scale_a.data_ptr()), max(1, scale_a.stride(0)),
        ctypes.c_void_p(scale_b.data_ptr()), max(1, scale_b.stride(0)), ctypes.c_void_p(cin),
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(wptr), wlen, ctypes.byref(c),
        ctypes.c_void_p(sp)))
    return out


MX6_FORMATS = {"e2m3": _abi.SK_MXF6E2M3, "e3m2": _abi.SK_MXF6E3M2}


def _mx6_problem(A, B, out, alpha, beta, fmt):
    """sk_problem of an MXFP6 product: A (M x 3K/4 bytes, row-major), B (3K/4
    x N bytes, column-major), out row-major M x N; sizes in elements."""
    if fmt not in MX6_FORMATS:
        raise ValueError(f"fmt must be one of {list(MX6_FORMATS)}")
    if A.dtype != torch.uint8 or B.dtype != torch.uint8:
        raise TypeError("MXFP6 operands: packed bytes (uint8)")
    if (A.numel() and A.stride(1) != 1) or (B.numel() and B.stride(0) != 1):
        raise ValueError("MXFP6: A row-major and B column-major")
    if A.shape[1] % 3 or B.shape[0] != A.shape[1]:
        raise ValueError("A and B must hold 3K/4 bytes of K per row / column")
    if A.stride(0) % 3 or B.stride(1) % 3:
        raise ValueError("row pitches must hold whole groups of four elements")
    M, K, N = A.shape[0], 4 * A.shape[1] // 3, B.shape[1]
    if tuple(out.shape) != (M, N) or out.dtype not in OUT_CODES or (out.stride(1) != 1 and N > 1):
        raise ValueError("out must be a row-major M x N float32/float16/bfloat16 tensor")
    return SkProblem(M, N, K, SK_ROW_MAJOR, SK_COL_MAJOR, max(4 * A.stride(0) // 3, K, 1),
                     max(4 * B.stride(1) // 3, K, 1), max(out.stride(0), N, 1), MX6_FORMATS[fmt],
                     OUT_CODES[out.dtype], alpha, beta, 1.0, 1.0)


def gemm_mx6(A, B, scale_a, scale_b, C=None, *, fmt="e2m3", alpha=1.0, beta=0.0, out=None,
             out_dtype=torch.float32, bias=None, activation="none", config=None,
             workspace=None, stream=None):
    """MXFP6 GEMM through sk_gemm_mx: A (M x 3K/4 bytes, row-major) and B
    (3K/4 x N bytes, column-major: the transpose of an N x 3K/4 row-major
    array) hold six-bit codes of `fmt` ("e2m3" or "e3m2"), element k of a
    row at bits 6k .. 6k+5 of its bytes read as one little-endian bit
    string; scale_a (M x >= K/32) and scale_b (N x >= K/32) hold one E8M0
    byte per 32 K-values, rows contiguous.
    out = act(alpha * sum_k (A * 2^(sa-127)) (B * 2^(sb-127)) + beta * C + bias)."""
    lib = load()
    if fmt not in MX6_FORMATS:
        raise ValueError(f"fmt must be one of {list(MX6_FORMATS)}")
    if A.dtype != torch.uint8 or B.dtype != torch.uint8:
        raise TypeError("MXFP6 operands: packed bytes (uint8)")
    for s_ in (scale_a, scale_b):
        if s_.dtype != torch.uint8 or s_.dim() != 2 or s_.stride(1) != 1 or not s_.is_cuda:
            raise TypeError("block scales: 2-D uint8 GPU tensors with contiguous rows")
    if not (A.is_cuda and B.is_cuda) or A.stride(1) != 1 or B.stride(0) != 1:
        raise ValueError("A row-major and B column-major on the GPU")
    if A.shape[1] % 3 or B.shape[0] != A.shape[1]:
        raise ValueError("A and B must hold 3K/4 bytes of K per row / column")
    M, K, N = A.shape[0], 4 * A.shape[1] // 3, B.shape[1]
    if out is None:
        out = C if (C is not None and beta != 0.0) else torch.empty(
            (M, N), dtype=out_dtype, device=A.device)
    if beta != 0.0 and C is None:
        raise ValueError("beta != 0 needs C")
    if scale_a.shape[0] != M or scale_b.shape[0] != N:
        raise ValueError("one scale row per row of A and per column of B")
    p = _set_epilogue(_mx6_problem(A, B, out, alpha, beta, fmt), bias, activation, A.device)
    if config is None:
        # the e4m3 rule (two steps per iteration) on the MX menu
        tile = default_tile(M, N, K, torch.float8_e4m3fn)
        config = Config(tile=(256, 128) if tile[0] == 256 else (128, 128))
    c = config.c_struct(MX6_FORMATS[fmt])
    sp = _stream_ptr(stream)
    nbytes = ctypes.c_size_t()
    check("sk_workspace_size", lib.sk_workspace_size(ctypes.byref(p), 1, ctypes.byref(c),
                                                      ctypes.byref(nbytes)))
    ws = workspace or workspace_for(A.device, sp)
    wptr, wlen = ws.get(nbytes.value, sp)
    cin = C.data_ptr() if (C is not None and beta != 0.0) else None
    check("sk_gemm_mx", lib.sk_gemm_mx(
        ctypes.byref(p), ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
        ctypes.c_void_p(scale_a.data_ptr()), max(1, scale_a.stride(0)),
        ctypes.c_void_p(scale_b.data_ptr()), max(1, scale_b.stride(0)), ctypes.c_void_p(cin),
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(wptr), wlen, ctypes.byref(c),
        ctypes.c_void_p(sp)))
    return out


def gemm_noalloc(A, B, C=None, *, alpha=1.0, beta=0.0, out=None, out_dtype=torch.float32,
                 scale_a=1.0, scale_b=1.0, bias=None, activation="none", config=None,
                 stream=None):
    """gemm() through sk_gemm_noalloc: the library's static per-GPU scratch
    array is the workspace, so the call allocates no device memory (with out
    given).  Calls that overlap on one GPU race; see include/streamk.h."""
    lib = load()
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("operands must be on the GPU")
    M, N = A.shape[0], B.shape[1]
    if out is None:
        out = C if (C is not None and beta != 0.0) else torch.empty(
            (M, N), dtype=out_dtype, device=A.device)
    if beta != 0.0 and C is None:
        raise ValueError("beta != 0 needs C")
    p = _set_epilogue(_problem(A, B, out, alpha, beta, scale_a, scale_b), bias, activation,
                      A.device)
    cfg = config or Config(tile=default_tile(M, N, A.shape[1], A.dtype))
    if C is not None and beta != 0.0:
        if tuple(C.shape) != (M, N) or C.dtype != out.dtype or C.stride() != out.stride():
            raise ValueError("C must match out in shape, dtype and strides")
    c = cfg.c_struct(p.dtype_ab)
    cin = C.data_ptr() if (C is not None and beta != 0.0) else None
    check("sk_gemm_noalloc", lib.sk_gemm_noalloc(
        ctypes.byref(p), ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
        ctypes.c_void_p(cin), ctypes.c_void_p(out.data_ptr()), ctypes.byref(c),
        ctypes.c_void_p(_stream_ptr(stream))))
    return out


def check_noalloc_error(stream=None):
    """Raise if a fixup wait of an earlier gemm_noalloc launch on this GPU
    timed out (reads and clears the scratch's error word)."""
    code = ctypes.c_int32()
    check("sk_check_device_error", load().sk_check_device_error(
        None, 0, ctypes.byref(code), ctypes.c_void_p(_stream_ptr(stream))))
    return code.value


def gemm_debug(A, B, *, out_dtype=torch.float32, config, partial_delay=0, reverse_ids=0,
               alpha=1.0, scale_a=1.0, scale_b=1.0, workspace=None):
    """gemm() through sk_gemm_debug: returns (out, segments, cover) where
    segments is the device trace of the segments each workgroup ran (list of
    tuples in SEGMENT_FIELDS order, sorted by workgroup, SK before DP, then
    tile) and cover[t][k] counts the runs of MAC iteration k of tile t."""
    lib = load()
    M, N = A.shape[0], B.shape[1]
    out = torch.empty((M, N), dtype=out_dtype, device=A.device)
    p = _problem(A, B, out, alpha, 0.0, scale_a, scale_b)
    c = config.c_struct(p.dtype_ab)
    info = SkPlanInfo()
    check("sk_plan", lib.sk_plan(ctypes.byref(p), 1, ctypes.byref(c), ctypes.byref(info)))
    cap = int(info.T) * 4 + int(info.g) * 4 + 16
    trace = torch.zeros((cap, 9), dtype=torch.int32, device=A.device)
    count = torch.zeros(1, dtype=torch.int64, device=A.device)
    stride = max(1, int(info.max_iters))
    cover = torch.zeros((max(1, int(info.T)), stride), dtype=torch.int32, device=A.device)
    dbg = SkDebug(trace.data_ptr(), cap, count.data_ptr(), cover.data_ptr(), stride,
                  partial_delay, reverse_ids)
    sp = _stream_ptr()
    ws = workspace or Workspace(A.device)
    wptr, wlen = ws.get(int(info.workspace_bytes), sp)
    check("sk_gemm_debug", lib.sk_gemm_debug(ctypes.byref(p), ctypes.c_void_p(A.data_ptr()),
                                             ctypes.c_void_p(B.data_ptr()), None,
                                             ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(wptr), wlen, ctypes.byref(c),
                                             ctypes.byref(dbg), ctypes.c_void_p(sp)))
    if wptr is not None:
        code = ctypes.c_int32()
        check("sk_check_device_error", lib.sk_check_device_error(
            ctypes.c_void_p(wptr), wlen, ctypes.byref(code), ctypes.c_void_p(sp)))
    torch.cuda.synchronize()
    n = int(count.item())
    if n > cap:
        raise RuntimeError(f"trace overflow: {n} segments > capacity {cap}")
    rows = [tuple(int(v) for v in r) for r in trace[:n].cpu().tolist()]
    rows.sort(key=lambda s: (s[0], s[7] == _abi.SK_ROLE_DP, s[2]))
    return out, rows, cover.cpu()


def check_device_error(workspace=None, stream=None):
    """Raise if a fixup wait of an earlier launch on this workspace timed out."""
    sp = _stream_ptr(stream)
    ws = workspace or workspace_for(torch.device("cuda", torch.cuda.current_device()), sp)
    if ws.buf is None:
        return 0
    code = ctypes.c_int32()
    check("sk_check_device_error", load().sk_check_device_error(
        ctypes.c_void_p(ws.buf.data_ptr()), ws.buf.numel(), ctypes.byref(code),
        ctypes.c_void_p(sp)))
    return code.value


# ---------------------------------------------------------------------------
# Host-only queries (no GPU needed when num_cu is given).

def _host_problem(M, N, K, dtype, layout_a="row", layout_b="col", beta=0.0):
    code = DTYPE_CODES[dtype] if isinstance(dtype, torch.dtype) else dtype
    la = SK_ROW_MAJOR if layout_a == "row" else SK_COL_MAJOR
    lb = SK_ROW_MAJOR if layout_b == "row" else SK_COL_MAJOR
    lda = max(1, K if la == SK_ROW_MAJOR else M)
    ldb = max(1, N if lb == SK_ROW_MAJOR else K)
    return SkProblem(M, N, K, la, lb, lda, ldb, max(1, N), code, _abi.SK_F32, 1.0, beta,
                     1.0, 1.0)


def _problems_array(shapes, dtype, beta=0.0):
    arr = (SkProblem * len(shapes))()
    for i, (M, N, K) in enumerate(shapes):
        arr[i] = _host_problem(M, N, K, dtype, beta=beta)
    return arr


def plan(shapes, dtype, config, beta=0.0):
    """Schedule parameters (dict) of problems [(M, N, K), ...] (beta: of
    every problem; it changes only the launch-time predictions)."""
    lib = load()
    probs = _problems_array(shapes, dtype, beta)
    c = config.c_struct(probs[0].dtype_ab)
    info = SkPlanInfo()
    check("sk_plan", lib.sk_plan(probs, len(shapes), ctypes.byref(c), ctypes.byref(info)))
    return {f: (float(getattr(info, f)) if f.startswith("predicted") else int(getattr(info, f)))
            for f, _ in SkPlanInfo._fields_}


def cost_model(dtype, tile):
    """Constants of the launch-time model the auto mode uses for (dtype,
    tile): a dict of t_launch, t_tile, t_it_full, t_it_light, t_store,
    t_peer (microseconds), l2, t_cin (microseconds), margin and the table
    row's tile."""
    code = DTYPE_CODES[dtype] if isinstance(dtype, torch.dtype) else dtype
    out = (ctypes.c_float * 10)()
    check("sk_cost_model", load().sk_cost_model(code, tile[0], tile[1], out, 10))
    names = ["t_launch", "t_tile", "t_it_full", "t_it_light", "t_store", "t_peer", "l2",
             "t_cin", "margin"]
    d = {n: float(v) for n, v in zip(names, out)}
    row = int(out[9])
    d["row_tile"] = (row // 65536, row % 65536)
    return d


def plan_order(shapes, dtype, config):
    """Caller indices of the problems in the order a launch concatenates them."""
    lib = load()
    probs = _problems_array(shapes, dtype)
    c = config.c_struct(probs[0].dtype_ab)
    out = (ctypes.c_int32 * len(shapes))()
    check("sk_plan_order", lib.sk_plan_order(probs, len(shapes), ctypes.byref(c), out))
    return list(out)


def launch_params(shapes, dtype, config):
    """The resolved launch parameters of a problem set, as the schedule
    simulator takes them: g, S, group_m, problem order, whether the launch
    is the data-parallel grid, and the rule that deals whole tiles."""
    info = plan(shapes, dtype, config)
    return {"g": info["g"], "S": info["S"], "group_m": info["group_m"],
            "order": plan_order(shapes, dtype, config), "dp_grid": bool(info["dp_grid"]),
            "deal": "serpentine"}


def schedule(shapes, dtype, config):
    """Full schedule from the library's host code: list of segment tuples."""
    lib = load()
    probs = _problems_array(shapes, dtype)
    c = config.c_struct(probs[0].dtype_ab)
    count = ctypes.c_int64()
    check("sk_schedule", lib.sk_schedule(probs, len(shapes), ctypes.byref(c), None, 0,
                                         ctypes.byref(count)))
    segs = (SkSegment * max(1, count.value))()
    check("sk_schedule", lib.sk_schedule(probs, len(shapes), ctypes.byref(c), segs,
                                         count.value, ctypes.byref(count)))
    return [tuple(getattr(segs[i], f) for f in SEGMENT_FIELDS) for i in range(count.value)]


def supported_tiles(dtype):
    lib = load()
    code = DTYPE_CODES[dtype] if isinstance(dtype, torch.dtype) else dtype
    n = ctypes.c_int32()
    check("sk_supported_tiles", lib.sk_supported_tiles(code, None, 0, ctypes.byref(n)))
    buf = (ctypes.c_int32 * (3 * n.value))()
    check("sk_supported_tiles", lib.sk_supported_tiles(code, buf, n.value, ctypes.byref(n)))
    return [(buf[3 * i], buf[3 * i + 1], buf[3 * i + 2]) for i in range(n.value)]


def device_query(config=None, dtype=torch.bfloat16):
    lib = load()
    cus = ctypes.c_int32()
    per = ctypes.c_int32()
    cfg = config or Config()
    c = cfg.c_struct(DTYPE_CODES[dtype])
    check("sk_device_query", lib.sk_device_query(ctypes.byref(cus), ctypes.byref(per),
                                                 ctypes.byref(c), DTYPE_CODES[dtype]))
    return cus.value, per.value


# ---------------------------------------------------------------------------
# Grouped GEMM.

class GroupedGemm:
    """One persistent Stream-K launch over several problems.

    problems: list of (A, B, out) or (A, B, out, C_in, beta) tuples sharing
    the input dtype, output dtype and operand layouts.  Descriptors and the
    workspace are set up once here (not capturable); run() only launches and
    can be captured into a HIP graph (torch.cuda.CUDAGraph).  biases: per
    problem a float32 vector of N values or None, added before the activation
    (one for every problem) in the fused epilogue.  mx_scales: MX problems
    (A, B torch.float8_e4m3fn codes for MXFP8, or packed bytes as for
    gemm_mx4 / gemm_mx6; A row-major, B column-major), per problem
    (scale_a, scale_b) as for gemm_mx; mx_format names the packed bytes'
    elements: "e2m1" (MXFP4, the default), "e2m3" or "e3m2" (MXFP6)."""

    def __init__(self, problems, config=None, alpha=1.0, scales=None, stream=None,
                 biases=None, activation="none", mx_scales=None, mx_format="e2m1"):
        lib = load()
        n = len(problems)
        if n == 0:
            raise ValueError("no problems")
        self.problems = problems
        self.biases = biases          # the descriptors hold their addresses
        probs = (SkProblem * n)()
        ptrs = {k: (ctypes.c_void_p * n)() for k in ("A", "B", "Cin", "Cout")}
        # the group's operand layouts, taken from its first non-empty operands
        nonempty_a = [p[0] for p in problems if p[0].numel() > 0]
        nonempty_b = [p[1] for p in problems if p[1].numel() > 0]
        prefer = (operand_layout(nonempty_a[0])[0] if nonempty_a else SK_ROW_MAJOR,
                  operand_layout(nonempty_b[0])[0] if nonempty_b else SK_COL_MAJOR)
        for i, pr in enumerate(problems):
            A, B, out = pr[:3]
            Cin = pr[3] if len(pr) > 3 else None
            beta = pr[4] if len(pr) > 4 else 0.0
            sa, sb = scales[i] if scales is not None else (1.0, 1.0)
            fp4 = mx_scales is not None and A.dtype in (torch.uint8, torch.float4_e2m1fn_x2)
            if fp4 and mx_format in MX6_FORMATS:
                base = _mx6_problem(A, B, out, alpha, beta, mx_format)
            elif fp4:
                if mx_format != "e2m1":
                    raise ValueError('mx_format must be "e2m1", "e2m3" or "e3m2"')
                base = _mx4_problem(A, B, out, alpha, beta)
            elif mx_scales is not None and A.dtype == torch.float8_e5m2:
                base = _problem(A.view(torch.float8_e4m3fn), B.view(torch.float8_e4m3fn), out,
                                alpha, beta, sa, sb, prefer)
            else:
                base = _problem(A, B, out, alpha, beta, sa, sb, prefer)
            probs[i] = _set_epilogue(base, biases[i] if biases is not None else None, activation,
                                     A.device)
            if mx_scales is not None and not fp4:
                if A.dtype not in MX8_CODES or B.dtype != A.dtype:
                    raise TypeError("MXFP8 operands: float8_e4m3fn or float8_e5m2 codes")
                probs[i].dtype_ab = MX8_CODES[A.dtype]
            ptrs["A"][i] = A.data_ptr()
            ptrs["B"][i] = B.data_ptr()
            ptrs["Cin"][i] = Cin.data_ptr() if (Cin is not None and beta != 0.0) else None
            ptrs["Cout"][i] = out.data_ptr()
        dev = problems[0][0].device
        M0, N0, K0 = probs[0].M, probs[0].N, probs[0].K
        if config is None:
            dt0 = (torch.bfloat16 if probs[0].dtype_ab == _abi.SK_MXF4E2M1 else
                   torch.float8_e4m3fn if probs[0].dtype_ab in MX6_FORMATS.values() or
                   probs[0].dtype_ab == _abi.SK_MXF8E5M2 else
                   problems[0][0].dtype)
            tile = default_tile(M0, N0, K0, dt0)
            if mx_scales is not None and tile not in ((256, 128), (128, 128)):
                tile = (256, 128) if tile[0] == 256 else (128, 128)   # the MX tile menu
            config = Config(tile=tile)
        self.config = config
        c = self.config.c_struct(probs[0].dtype_ab)
        dbytes = ctypes.c_size_t()
        check("sk_grouped_desc_size", lib.sk_grouped_desc_size(n, ctypes.byref(dbytes)))
        self.desc = torch.empty(dbytes.value, dtype=torch.uint8, device=dev)
        self.plan = SkGroupedPlan()
        sp = _stream_ptr(stream)
        if mx_scales is None:
            check("sk_grouped_prepare", lib.sk_grouped_prepare(
                probs, ptrs["A"], ptrs["B"], ptrs["Cin"], ptrs["Cout"], n, ctypes.byref(c),
                ctypes.c_void_p(self.desc.data_ptr()), dbytes.value, ctypes.byref(self.plan),
                ctypes.c_void_p(sp)))
        else:
            if len(mx_scales) != n:
                raise ValueError("one (scale_a, scale_b) pair per problem")
            self.mx_scales = mx_scales    # the descriptors hold their addresses
            sp_a, sp_b = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)()
            ld_a, ld_b = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
            for i, (s_a, s_b) in enumerate(mx_scales):
                for t in (s_a, s_b):
                    if t.dtype != torch.uint8 or t.dim() != 2 or t.stride(1) != 1 or not t.is_cuda:
                        raise TypeError("block scales: 2-D uint8 GPU tensors with contiguous rows")
                sp_a[i], ld_a[i] = s_a.data_ptr(), max(1, s_a.stride(0))
                sp_b[i], ld_b[i] = s_b.data_ptr(), max(1, s_b.stride(0))
            check("sk_grouped_prepare_mx", lib.sk_grouped_prepare_mx(
                probs, ptrs["A"], ptrs["B"], sp_a, ld_a, sp_b, ld_b, ptrs["Cin"], ptrs["Cout"], n,
                ctypes.byref(c), ctypes.c_void_p(self.desc.data_ptr()), dbytes.value,
                ctypes.byref(self.plan), ctypes.c_void_p(sp)))
        self.workspace = Workspace(dev)
        self.ws_ptr, self.ws_len = self.workspace.get(int(self.plan.workspace_bytes), sp)
        torch.cuda.current_stream().synchronize()

    def info(self):
        return {f: int(getattr(self.plan, f)) for f, _ in SkGroupedPlan._fields_}

    def run(self, stream=None):
        check("sk_gemm_grouped", load().sk_gemm_grouped(
            ctypes.byref(self.plan), ctypes.c_void_p(self.desc.data_ptr()),
            ctypes.c_void_p(self.ws_ptr), self.ws_len, ctypes.c_void_p(_stream_ptr(stream))))

    def run_debug(self, partial_delay=0, reverse_ids=0):
        """run() through sk_gemm_grouped_debug: returns (segments, cover) as
        gemm_debug does (segment problem = the caller's index)."""
        lib = load()
        dev = self.desc.device
        T, g = int(self.plan.T), int(self.plan.g)
        cap = T * 4 + g * 4 + 16
        trace = torch.zeros((cap, 9), dtype=torch.int32, device=dev)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        stride = max(1, int(self.plan.max_iters))
        cover = torch.zeros((max(1, T), stride), dtype=torch.int32, device=dev)
        dbg = SkDebug(trace.data_ptr(), cap, count.data_ptr(), cover.data_ptr(), stride,
                      partial_delay, reverse_ids)
        sp = _stream_ptr()
        check("sk_gemm_grouped_debug", lib.sk_gemm_grouped_debug(
            ctypes.byref(self.plan), ctypes.c_void_p(self.desc.data_ptr()),
            ctypes.c_void_p(self.ws_ptr), self.ws_len, ctypes.byref(dbg), ctypes.c_void_p(sp)))
        if self.ws_ptr is not None:
            code = ctypes.c_int32()
            check("sk_check_device_error", lib.sk_check_device_error(
                ctypes.c_void_p(self.ws_ptr), self.ws_len, ctypes.byref(code),
                ctypes.c_void_p(sp)))
        torch.cuda.synchronize()
        n = int(count.item())
        if n > cap:
            raise RuntimeError(f"trace overflow: {n} segments > capacity {cap}")
        rows = [tuple(int(v) for v in r) for r in trace[:n].cpu().tolist()]
        rows.sort(key=lambda s: (s[0], s[7] == _abi.SK_ROLE_DP, s[2]))
        return rows, cover.cpu()

    def capture(self):
        """A torch.cuda.CUDAGraph (a HIP graph on ROCm) holding one run()."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()   # warm-up launch outside the graph
        torch.cuda.current_stream().wait_stream(s)
        with torch.cuda.graph(g):
            self.run()
        return g


# ---------------------------------------------------------------------------
# Differentiable linear layer.

def transpose(t, stream=None):
    """Row-major transposed copy of a row-major 2-D GPU tensor through
    sk_transpose: u[j, i] = t[i, j], bit for bit (1-, 2- and 4-byte
    elements)."""
    if t.dim() != 2 or not t.is_cuda:
        raise ValueError("transpose: a 2-D GPU tensor")
    rows, cols = t.shape
    if t.numel() and t.stride(1) != 1 and cols > 1:
        raise ValueError("transpose: rows must be contiguous (unit column stride)")
    eb = t.element_size()
    u = torch.empty((cols, rows), dtype=t.dtype, device=t.device)
    check("sk_transpose", load().sk_transpose(
        ctypes.c_void_p(t.data_ptr()), rows, cols, max(1, t.stride(0), cols),
        ctypes.c_void_p(u.data_ptr()), max(1, rows), eb, ctypes.c_void_p(_stream_ptr(stream))))
    return u


def k_contiguous(op, role, stream=None):
    """`op` itself if its K dimension is contiguous, else a K-contiguous copy
    (sk_transpose): role "a" for an M x K operand (K-contiguous = row-major),
    "b" for a K x N operand (K-contiguous = column-major)."""
    if role == "a":
        if op.stride(1) == 1 or op.shape[1] <= 1:
            return op
        return transpose(op.t(), stream)    # op.t() is K x M row-major
    if op.stride(0) == 1 or op.shape[0] <= 1:
        return op
    return transpose(op, stream).t()        # N x K row-major, viewed K x N


def pack_pays(M, N, K, dtype):
    """Whether a product with M- or N-major operands should be computed from
    K-contiguous copies.  Transposing LDS reads cost the 16-bit and e4m3
    kernels up to 30-45% (BF16 1024x4096x4096 with both operands M/N-major:
    70.8 us as laid out, 50.9 us packed, copies included), while a copy moves
    each operand byte twice at 5-7 TB/s; the copies lose where K is short
    (BF16 4096x4096x1024, A M-major and B N-major: 0.90x) or the product is
    small (1024^3: 0.84-1.02x; e4m3, whose GEMMs are faster, 2048^3: 0.76-0.91x).
    Measured on 8 shapes x 3 layouts per type: K >= 2048 and M*N >= 2^22
    (and M*N*K >= 2^35 for e4m3) packs every product that gains and none that
    loses more than 1%."""
    code = DTYPE_CODES[dtype] if isinstance(dtype, torch.dtype) else dtype
    if code not in (_abi.SK_F16, _abi.SK_BF16, _abi.SK_F8E4M3, _abi.SK_F8E5M2):
        return False
    if K < 2048 or M * N < (1 << 22):
        return False
    return code not in (_abi.SK_F8E4M3, _abi.SK_F8E5M2) or M * N * K >= (1 << 35)


class StreamKLinearFn(torch.autograd.Function):
    """Y = X @ W^T with a hand-written backward through the same kernels:
    dX = dY @ W and dW = dY^T @ X.  The forward reads W as a column-major
    K x N operand (K-contiguous, no copy).  The backward products take W, dY
    and X as laid out (B N-major for dX; A M-major and B N-major for dW), or,
    with `pack` (True, or "auto": when pack_pays), K-contiguous copies made by
    sk_transpose."""

    @staticmethod
    def forward(ctx, X, W, config_fwd=None, config_dx=None, config_dw=None, pack="auto"):
        ctx.save_for_backward(X, W)
        ctx.cfgs = (config_dx, config_dw)
        ctx.pack = pack
        Y = torch.empty((X.shape[0], W.shape[0]), dtype=X.dtype, device=X.device)
        return gemm(X, W.t(), out=Y, config=config_fwd)

    @staticmethod
    def backward(ctx, dY):
        X, W = ctx.saved_tensors
        cfg_dx, cfg_dw = ctx.cfgs
        if dY.stride(1) != 1 and dY.stride(0) != 1:
            dY = dY.contiguous()

        def packed(M, N, K):
            return ctx.pack is True or (ctx.pack == "auto" and pack_pays(M, N, K, X.dtype))

        dX = dW = None
        if ctx.needs_input_grad[0]:
            dX = torch.empty_like(X, memory_format=torch.contiguous_format)
            B = W
            if packed(dY.shape[0], W.shape[1], W.shape[0]):
                B = k_contiguous(W, "b")
            gemm(dY, B, out=dX, config=cfg_dx)
        if ctx.needs_input_grad[1]:
            dW = torch.empty_like(W, memory_format=torch.contiguous_format)
            A, B = dY.t(), X
            if packed(W.shape[0], W.shape[1], X.shape[0]):
                A, B = k_contiguous(A, "a"), k_contiguous(B, "b")
            gemm(A, B, out=dW, config=cfg_dw)
        return dX, dW, None, None, None, None


def linear(X, W, config_fwd=None, config_dx=None, config_dw=None, pack="auto"):
    """Y = X @ W^T (StreamKLinearFn); `pack`: True, False or "auto", whether
    the backward products read K-contiguous copies of their operands."""
    if pack not in (True, False, "auto"):
        raise ValueError('pack must be True, False or "auto"')
    return StreamKLinearFn.apply(X, W, config_fwd, config_dx, config_dw, pack)


def with_tile(config, tile):
    return replace(config, tile=tuple(tile))
