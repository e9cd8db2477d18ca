"""Seeded synthetic inputs shared by the tests and the benchmark.

Holds no GEMM arithmetic: it only draws numbers (numpy PCG64 streams in
float64), rounds them to the input type with torch's round-to-nearest-even
conversions, and places matrices in memory with a requested layout and
leading dimension.  Both the GPU path and the oracle consume what this
module produces; neither is imported here.
"""
import math

import numpy as np
import torch

E4M3_MAX = 448.0   # largest finite OCP e4m3fn value

TORCH_DTYPES = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16,
                "e4m3": torch.float8_e4m3fn, "e5m2": torch.float8_e5m2}
CODE_VIEW = {"f32": (torch.int32, np.uint32), "f16": (torch.int16, np.uint16),
             "bf16": (torch.int16, np.uint16), "e4m3": (torch.uint8, np.uint8),
             "e5m2": (torch.uint8, np.uint8)}


def rng(seed):
    return np.random.default_rng(seed)


def uniform(shape, seed, lo=-1.0, hi=1.0):
    return rng(seed).uniform(lo, hi, size=shape)


def normal(shape, seed):
    return rng(seed).standard_normal(size=shape)


def integers(shape, seed, lo=-4, hi=4):
    """Uniform over the integers lo..hi inclusive, as float64."""
    return rng(seed).integers(lo, hi + 1, size=shape).astype(np.float64)


def round_to(x64, dtype):
    """float64 array -> CPU torch tensor of `dtype` ('f32','f16','bf16')."""
    return torch.from_numpy(np.ascontiguousarray(x64)).to(TORCH_DTYPES[dtype])


def fp8_scaled(x64, elem="e4m3"):
    """Per-tensor amax scaling into the e4m3fn range (elem="e5m2": the e5m2
    range).

    scale = max|x| / emax (as a float32; emax 448, e5m2 57344), q = RNE(x /
    scale) in the element format; |q| <= emax by construction, so nothing
    saturates.  Returns (q tensor, scale float)."""
    tdtype, emax = _MX8[elem]
    amax = float(np.max(np.abs(x64))) if x64.size else 0.0
    scale = float(np.float32(amax / emax)) if amax > 0 else 1.0
    q = torch.from_numpy(np.ascontiguousarray(x64 / scale)).to(tdtype)
    return q, scale


E5M2_MAX = 57344.0   # largest finite OCP e5m2 value
_MX8 = {"e4m3": (torch.float8_e4m3fn, E4M3_MAX), "e5m2": (torch.float8_e5m2, E5M2_MAX)}


def mx_quantize(x64, block=32, elem="e4m3"):
    """MX quantisation of rows along K: for each block of `block` consecutive
    K-values of a row, the shared exponent X = ceil(log2(amax / emax)) (the
    smallest power of two that brings the block into the element range, so
    nothing saturates; emax 448 for e4m3, 57344 for e5m2; amax 0 gives
    X = 0) is stored as the E8M0 code X + 127, and the elements become
    RNE(x / 2^X) in the element format.  Returns (codes tensor R x K, uint8
    scale array R x ceil(K/block))."""
    tdtype, E4M3_MAX = _MX8[elem]   # noqa: N806 (the element format's max)
    x = np.asarray(x64, dtype=np.float64)
    R, K = x.shape
    nb = -(-K // block)
    e = np.zeros((R, nb), dtype=np.int64)
    q = np.empty_like(x)
    for b in range(nb):
        blk = x[:, b * block:(b + 1) * block]
        amax = np.max(np.abs(blk), axis=1)
        safe = np.where(amax > 0, amax, E4M3_MAX)
        X = np.ceil(np.log2(safe / E4M3_MAX))
        # guard the log's rounding: the smallest X with amax / 2^X <= 448
        X = np.where(safe / np.ldexp(1.0, X.astype(np.int64)) > E4M3_MAX, X + 1, X)
        X = np.where(safe / np.ldexp(1.0, (X - 1).astype(np.int64)) <= E4M3_MAX, X - 1, X)
        X = np.clip(np.where(amax > 0, X, 0), -127, 127).astype(np.int64)
        e[:, b] = X + 127
        q[:, b * block:(b + 1) * block] = np.clip(blk / np.ldexp(1.0, X)[:, None], -E4M3_MAX,
                                                  E4M3_MAX)
    codes_t = torch.from_numpy(np.ascontiguousarray(q)).to(tdtype)
    return codes_t, e.astype(np.uint8)


FP4_MAX = 6.0
# E2M1 magnitudes of codes 0..7 and the midpoints between neighbours
_FP4_GRID = np.array([0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0])
_FP4_MID = (_FP4_GRID[:-1] + _FP4_GRID[1:]) / 2


def fp4_rne(x):
    """Round to the nearest E2M1 (FP4) value, ties to the code with an even
    mantissa, saturating at +-6: returns 4-bit codes (int64)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), FP4_MAX)
    idx = np.zeros(a.shape, dtype=np.int64)
    for i, m in enumerate(_FP4_MID):
        # a tie between codes i and i+1 goes to the even one
        idx += (a > m) if i % 2 == 0 else (a >= m)
    return idx | (np.signbit(x).astype(np.int64) << 3)


def pack_fp4(codes4):
    """4-bit codes R x K (K even) -> bytes R x K/2, element 2j in the low
    nibble of byte j."""
    c = np.asarray(codes4, dtype=np.int64)
    return (c[:, 0::2] | (c[:, 1::2] << 4)).astype(np.uint8)


def mx4_quantize(x64, block=32):
    """MXFP4 quantisation of rows along K: for each block of `block`
    consecutive K-values of a row, the shared exponent X = the smallest power
    of two with amax / 2^X <= 6 (amax 0 gives X = 0) is stored as the E8M0
    code X + 127, and the elements become the nearest E2M1 value of x / 2^X.
    Returns (packed FP4 bytes R x K/2, uint8 scale array R x ceil(K/block))."""
    x = np.asarray(x64, dtype=np.float64)
    R, K = x.shape
    nb = -(-K // block)
    e = np.zeros((R, nb), dtype=np.int64)
    c = np.empty(x.shape, dtype=np.int64)
    for b in range(nb):
        blk = x[:, b * block:(b + 1) * block]
        amax = np.max(np.abs(blk), axis=1)
        safe = np.where(amax > 0, amax, FP4_MAX)
        X = np.ceil(np.log2(safe / FP4_MAX))
        X = np.where(safe / np.ldexp(1.0, X.astype(np.int64)) > FP4_MAX, X + 1, X)
        X = np.where(safe / np.ldexp(1.0, (X - 1).astype(np.int64)) <= FP4_MAX, X - 1, X)
        X = np.clip(np.where(amax > 0, X, 0), -127, 127).astype(np.int64)
        e[:, b] = X + 127
        c[:, b * block:(b + 1) * block] = fp4_rne(blk / np.ldexp(1.0, X)[:, None])
    return pack_fp4(c), e.astype(np.uint8)


FP6_MAX = {"e2m3": 7.5, "e3m2": 28.0}
_FP6_FIELDS = {"e2m3": (2, 3, 1), "e3m2": (3, 2, 3)}   # exponent bits, mantissa bits, bias


def _fp6_grid(fmt):
    """Non-negative FP6 magnitudes in code order (codes 0..31)."""
    eb, mb, bias = _FP6_FIELDS[fmt]
    out = []
    for c in range(32):
        e, m = c >> mb, c & ((1 << mb) - 1)
        out.append(math.ldexp(m, 1 - bias - mb) if e == 0 else
                   math.ldexp((1 << mb) + m, e - bias - mb))
    return np.array(out)


def fp6_rne(x, fmt):
    """Round to the nearest FP6 value of `fmt` ("e2m3" or "e3m2"), ties to
    the code with an even mantissa, saturating at the largest magnitude:
    returns 6-bit codes (int64)."""
    grid = _fp6_grid(fmt)
    mid = (grid[:-1] + grid[1:]) / 2
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), grid[-1])
    idx = np.zeros(a.shape, dtype=np.int64)
    for i, m in enumerate(mid):
        # a tie between codes i and i+1 goes to the even one
        idx += (a > m) if i % 2 == 0 else (a >= m)
    return idx | (np.signbit(x).astype(np.int64) << 5)


def pack_fp6(codes6):
    """6-bit codes R x K (K a multiple of 4) -> bytes R x 3K/4, element k at
    bits 6k .. 6k+5 of the row's little-endian bit string."""
    c = np.asarray(codes6, dtype=np.int64)
    R, K = c.shape
    g = c.reshape(R, K // 4, 4)
    word = g[..., 0] | (g[..., 1] << 6) | (g[..., 2] << 12) | (g[..., 3] << 18)   # 24 bits
    out = np.stack([word & 255, (word >> 8) & 255, (word >> 16) & 255], axis=-1)
    return out.reshape(R, 3 * K // 4).astype(np.uint8)


def mx6_quantize(x64, fmt, block=32):
    """MXFP6 quantisation of rows along K: for each block of `block`
    consecutive K-values of a row, the shared exponent X = the smallest
    power of two with amax / 2^X <= the format's largest value (amax 0 gives
    X = 0) is stored as the E8M0 code X + 127, and the elements become the
    nearest FP6 value of x / 2^X.  Returns (packed bytes R x 3K/4, uint8
    scale array R x ceil(K/block))."""
    x = np.asarray(x64, dtype=np.float64)
    top = FP6_MAX[fmt]
    R, K = x.shape
    nb = -(-K // block)
    e = np.zeros((R, nb), dtype=np.int64)
    c = np.empty(x.shape, dtype=np.int64)
    for b in range(nb):
        blk = x[:, b * block:(b + 1) * block]
        amax = np.max(np.abs(blk), axis=1)
        safe = np.where(amax > 0, amax, top)
        X = np.ceil(np.log2(safe / top))
        X = np.where(safe / np.ldexp(1.0, X.astype(np.int64)) > top, X + 1, X)
        X = np.where(safe / np.ldexp(1.0, (X - 1).astype(np.int64)) <= top, X - 1, X)
        X = np.clip(np.where(amax > 0, X, 0), -127, 127).astype(np.int64)
        e[:, b] = X + 127
        c[:, b * block:(b + 1) * block] = fp6_rne(blk / np.ldexp(1.0, X)[:, None], fmt)
    return pack_fp6(c), e.astype(np.uint8)


def codes(t):
    """Raw bit patterns of a CPU tensor (uint32/uint16/uint8 numpy array)."""
    dt = {v: k for k, v in TORCH_DTYPES.items()}[t.dtype]
    tv, nv = CODE_VIEW[dt]
    return t.contiguous().view(tv).numpy().view(nv)


def place(t, col_major=False, ld=None, device=None, fill=0):
    """Put logical matrix t (rows x cols) in storage with the given layout.

    Row-major: storage (rows, ld), ld >= cols, element (i, j) at i*ld + j.
    Column-major: storage (cols, ld), ld >= rows, element (i, j) at j*ld + i.
    Returns (view, storage, ld): `view` has t's shape and the layout's
    strides; padding elements of the storage hold `fill` (as codes 0 unless
    given)."""
    rows, cols = t.shape
    inner = rows if col_major else cols
    ld = max(1, inner) if ld is None else ld
    if ld < inner:
        raise ValueError("leading dimension smaller than the matrix extent")
    outer = cols if col_major else rows
    store = torch.full((outer, ld), fill, dtype=t.dtype) \
        if t.dtype not in (torch.float8_e4m3fn, torch.float8_e5m2) \
        else torch.zeros((outer, ld), dtype=torch.uint8).view(t.dtype)
    if col_major:
        store[:, :rows] = t.t()
    else:
        store[:, :cols] = t
    if device is not None:
        store = store.to(device)
    view = store[:, :rows].t() if col_major else store[:, :cols]
    return view, store, ld


def ld_aligned(extent, elem_bytes, align=16):
    """Smallest leading dimension >= extent whose row is a multiple of
    `align` bytes (storage padding only; the problem keeps its size)."""
    per = align // math.gcd(align, elem_bytes)
    return max(per, -(-extent // per) * per)


def log_uniform_int(r, lo, hi):
    return int(round(math.exp(r.uniform(math.log(lo), math.log(hi)))))


def sweep_shapes(seed=3, n=64):
    """64 shapes, M,N log-uniform in [128, 8192], K log-uniform in
    [128, 16384] (BF16 shape sweep)."""
    r = rng(seed)
    return [(log_uniform_int(r, 128, 8192), log_uniform_int(r, 128, 8192),
             log_uniform_int(r, 128, 16384)) for _ in range(n)]


def grouped_shapes(seed=5, n=48):
    """48 problems, M log-uniform in [16, 4096], N in {1024, 2048, 4096},
    K in {2048, 4096, 8192} (grouped FP8 set)."""
    r = rng(seed)
    out = []
    for _ in range(n):
        m = log_uniform_int(r, 16, 4096)
        nn = int(r.choice([1024, 2048, 4096]))
        k = int(r.choice([2048, 4096, 8192]))
        out.append((m, nn, k))
    return out
