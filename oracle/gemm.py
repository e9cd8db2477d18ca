"""FP64 reference GEMM and exact input decoders -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
use this module (see the package docstring).

The report frames the whole study around the general matrix product
(Introduction; Background) and measures it as C = A*B on square and irregular
shapes (Results, Table 1).  Stream-K changes only how the multiply-accumulate
work is distributed, so -- up to floating-point summation order -- it must
reach exactly the plain product.  The oracle is therefore that plain product,

    C[i][j] = alpha * s_A * s_B * sum_k A(i,k) B(k,j) + beta * Cin[i][j],

evaluated in IEEE double on the *same rounded inputs* the GPU receives: the
bf16 / f16 / e4m3fn / f32 codes are decoded exactly to float64 by the decoders
below, which are written from the published bit-level format definitions, not
from any library conversion routine.  ``s_A``, ``s_B`` are the per-tensor
scales of FP8 inputs (1 otherwise).  MXFP8 inputs (OCP MX block scaling)
multiply each block of 32 K-values of a row of A or a column of B by a
power-of-two E8M0 scale first (gemm_mx), which is exact in FP64.  The
fused epilogue (bias per output column, then an activation) is applied to
that FP64 result by ``epilogue``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_gemm_f64.argtypes = [i64, i64, i64, p, i64, ctypes.c_int,
                                        p, i64, ctypes.c_int, p, i64,
                                        ctypes.c_double, ctypes.c_double,
                                        p, i64, p, i64]
        lib.oracle_gemm_f64.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    """OpenMP threads the C oracle uses for one call."""
    return int(_load().oracle_num_threads())


# ---------------------------------------------------------------------------
# Exact decoders, written from the format definitions.
#
# A binary floating-point code with sign bit s, an e-bit biased exponent E and
# an m-bit fraction F encodes
#     (-1)^s * 2^(E - bias) * (1 + F / 2^m)      for 0 < E < E_max  (normal)
#     (-1)^s * 2^(1 - bias) * (F / 2^m)          for E == 0         (subnormal)
# bfloat16: e=8, m=7, bias=127 (IEEE binary32 truncated to 16 bits); E=255 is
#           inf (F=0) or NaN.
# float16 : e=5, m=10, bias=15 (IEEE binary16); E=31 is inf (F=0) or NaN.
# e4m3fn  : e=4, m=3, bias=7 (OCP 8-bit float, "fn" = finite): there is no
#           infinity; only S.1111.111 is NaN, so E=15 with F<7 is a normal
#           number and the largest finite value is 1.75 * 2^8 = 448.
# Every value of these formats is exactly representable in float64, so the
# decode is exact; it is evaluated with numpy.ldexp on integers, which is an
# exact power-of-two scaling.
# ---------------------------------------------------------------------------

def _decode_fields(code, ebits, mbits, bias):
    code = np.asarray(code).astype(np.int64)
    sign = (code >> (ebits + mbits)) & 1
    e = (code >> mbits) & ((1 << ebits) - 1)
    f = code & ((1 << mbits) - 1)
    normal = np.ldexp((1 << mbits) + f, (e - bias - mbits).astype(np.int32))
    subnormal = np.ldexp(f.astype(np.float64), 1 - bias - mbits)
    mag = np.where(e == 0, subnormal, normal).astype(np.float64)
    return sign, e, f, np.where(sign == 1, -mag, mag)


def decode_bf16(bits) -> np.ndarray:
    """uint16 bfloat16 codes -> exact float64 values."""
    sign, e, f, v = _decode_fields(bits, 8, 7, 127)
    special = e == 255
    v = np.where(special & (f == 0), np.where(sign == 1, -np.inf, np.inf), v)
    return np.where(special & (f != 0), np.nan, v)


def decode_f16(bits) -> np.ndarray:
    """uint16 IEEE binary16 codes -> exact float64 values."""
    sign, e, f, v = _decode_fields(bits, 5, 10, 15)
    special = e == 31
    v = np.where(special & (f == 0), np.where(sign == 1, -np.inf, np.inf), v)
    return np.where(special & (f != 0), np.nan, v)


def decode_e4m3fn(bits) -> np.ndarray:
    """uint8 OCP e4m3fn codes -> exact float64 values."""
    sign, e, f, v = _decode_fields(bits, 4, 3, 7)
    return np.where((e == 15) & (f == 7), np.nan, v)


def decode_e5m2(bits) -> np.ndarray:
    """uint8 OCP e5m2 codes -> exact float64 values: sign bit, 5 exponent
    bits with bias 15, 2 mantissa bits; exponent 31 encodes infinity
    (mantissa 0) and NaN (otherwise), as in IEEE binary16, whose upper byte
    it is."""
    sign, e, f, v = _decode_fields(bits, 5, 2, 15)
    special = e == 31
    v = np.where(special & (f == 0), np.where(sign == 1, -np.inf, np.inf), v)
    return np.where(special & (f != 0), np.nan, v)


def decode_f32(bits) -> np.ndarray:
    """uint32 IEEE binary32 codes -> exact float64 values (the widening of
    binary32 to binary64 is exact)."""
    return np.ascontiguousarray(bits, dtype=np.uint32).view(np.float32).astype(np.float64)


def decode_e8m0(bits) -> np.ndarray:
    """uint8 OCP E8M0 scale codes -> exact float64 values.  E8M0 is an
    8-bit biased exponent alone (no sign, no fraction): code e encodes
    2^(e - 127) for e = 0..254, and e = 255 is NaN."""
    e = np.asarray(bits).astype(np.int64)
    v = np.ldexp(np.ones(e.shape, dtype=np.float64), (e - 127).astype(np.int32))
    return np.where(e == 255, np.nan, v)


def decode_e2m1(bits) -> np.ndarray:
    """4-bit OCP FP4 (E2M1) codes 0..15 -> exact float64 values: sign bit,
    2 exponent bits with bias 1, 1 mantissa bit; exponent 0 is subnormal
    (0.5 * m); no infinities or NaN, so the magnitudes are 0, 0.5, 1, 1.5,
    2, 3, 4 and 6."""
    _, _, _, v = _decode_fields(np.asarray(bits).astype(np.int64) & 15, 2, 1, 1)
    return v


def unpack_fp4(packed, count) -> np.ndarray:
    """Packed FP4 bytes -> `count` codes: element 2j in the low nibble of byte
    j, element 2j+1 in the high nibble."""
    b = np.asarray(packed).astype(np.int64).reshape(-1)
    codes = np.empty(2 * b.size, dtype=np.int64)
    codes[0::2] = b & 15
    codes[1::2] = b >> 4
    return codes[:count]


def decode_e2m3(bits) -> np.ndarray:
    """6-bit OCP FP6 E2M3 codes 0..63 -> exact float64 values: sign bit, 2
    exponent bits with bias 1, 3 mantissa bits; exponent 0 is subnormal
    (m / 8); no infinities or NaN, so the largest magnitude is 7.5."""
    _, _, _, v = _decode_fields(np.asarray(bits).astype(np.int64) & 63, 2, 3, 1)
    return v


def decode_e3m2(bits) -> np.ndarray:
    """6-bit OCP FP6 E3M2 codes 0..63 -> exact float64 values: sign bit, 3
    exponent bits with bias 3, 2 mantissa bits; exponent 0 is subnormal
    (m / 16); no infinities or NaN, so the largest magnitude is 28."""
    _, _, _, v = _decode_fields(np.asarray(bits).astype(np.int64) & 63, 3, 2, 3)
    return v


def unpack_fp6(packed, count) -> np.ndarray:
    """Packed FP6 bytes -> `count` codes: element k at bits 6k .. 6k+5 of
    the bytes read as one little-endian bit string (four elements in three
    bytes: byte 3j holds element 4j and the low 2 bits of element 4j+1, ...)."""
    b = np.asarray(packed).astype(np.int64).reshape(-1)
    bits = ((b[:, None] >> np.arange(8)) & 1).reshape(-1)      # bit 8i+t of the string
    n = min(count, bits.size // 6)
    w = bits[:6 * n].reshape(n, 6)
    return (w << np.arange(6)).sum(axis=1)


DECODERS = {"f32": decode_f32, "f16": decode_f16, "bf16": decode_bf16,
            "e4m3": decode_e4m3fn}


def decode(dtype: str, bits) -> np.ndarray:
    """Decode raw codes of an input dtype ('f32', 'f16', 'bf16', 'e4m3')."""
    return DECODERS[dtype](bits)


# ---------------------------------------------------------------------------
# The product.
# ---------------------------------------------------------------------------

def gemm(M, N, K, a, lda, a_col_major, b, ldb, b_col_major, alpha=1.0,
         beta=0.0, cin=None, ldcin=None, rows=None):
    """C = alpha * A*B + beta * Cin in float64 (plain definition, C loop).

    ``a``/``b`` are float64 storage arrays indexed as documented in
    gemm_f64.c (row-major: x[i*ld + k]; column-major: x[k*ld + i]).
    ``alpha`` is the full output scale (alpha * s_A * s_B for FP8).
    ``rows``: optional list of output rows to compute (row sample).
    Returns a (len(rows) or M) x N float64 array.
    """
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    if rows is not None:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nout = rows.size
    else:
        nout = M
    out = np.empty((max(nout, 0), max(N, 0)), dtype=np.float64)
    if beta != 0.0:
        cin = np.ascontiguousarray(cin, dtype=np.float64).reshape(-1)
        cin_p = cin.ctypes.data
        if ldcin is None:
            ldcin = N
    else:
        cin_p = None
        ldcin = 0
    if nout == 0 or N == 0:
        return out
    rc = lib.oracle_gemm_f64(M, N, K, a.ctypes.data if a.size else None, lda,
                             int(a_col_major),
                             b.ctypes.data if b.size else None, ldb,
                             int(b_col_major), cin_p, ldcin,
                             float(alpha), float(beta), out.ctypes.data, N,
                             rows.ctypes.data if rows is not None else None,
                             nout)
    if rc != 0:
        raise ValueError(f"oracle_gemm_f64 failed with code {rc}")
    return out


def mx_operand(codes, ld, scales, ld_s, rows, K, block=32, elem="e4m3"):
    """An MX operand stored K-contiguous (OCP MX block scaling): element
    (r, k) is decode(codes[r*ld + k]) * decode_e8m0(scales[r*ld_s +
    k // block]), the elements e4m3 codes (elem="e5m2": e5m2 codes), or
    with elem="e2m1" FP4 codes or
    elem="e2m3" / "e3m2" FP6 codes unpacked from bytes (ld then counts
    elements: row r starts at element r*ld).  Returns the rows x K float64 values; each is a decoded element
    times a power of two, so the result is exact."""
    if elem == "e2m1":
        x = decode_e2m1(unpack_fp4(codes, 2 * np.asarray(codes).size))
    elif elem in ("e2m3", "e3m2"):
        c = unpack_fp6(codes, 8 * np.asarray(codes).size // 6)
        x = decode_e2m3(c) if elem == "e2m3" else decode_e3m2(c)
    elif elem == "e5m2":
        x = decode_e5m2(np.asarray(codes).reshape(-1))
    else:
        x = decode_e4m3fn(np.asarray(codes).reshape(-1))
    s = decode_e8m0(np.asarray(scales).reshape(-1))
    out = np.empty((rows, K), dtype=np.float64)
    for r in range(rows):
        blk = s[r * ld_s + np.arange(K) // block]
        out[r] = x[r * ld: r * ld + K] * blk
    return out


def gemm_mx(M, N, K, a_codes, lda, sa, ldsa, b_codes, ldb, sb, ldsb, alpha=1.0, beta=0.0,
            cin=None, rows=None, elem="e4m3"):
    """MX product C = alpha * sum_k A^(i,k) B^(k,j) + beta * Cin, with A
    row-major (row i at a_codes[i*lda]) and B column-major (column j at
    b_codes[j*ldb]) element codes (e4m3 or e5m2 bytes, or with elem="e2m1" FP4
    codes packed two per byte, lda/ldb counted in elements) and E8M0 scales
    of every 32 K-values of each row of A (sa[i*ldsa + k//32]) and column of
    B (sb[j*ldsb + k//32]): A^ and B^ are the block-scaled values
    (mx_operand, exact), multiplied by the plain FP64 product above."""
    ahat = mx_operand(a_codes, lda, sa, ldsa, M, K, elem=elem)
    bhat_t = mx_operand(b_codes, ldb, sb, ldsb, N, K, elem=elem)   # row j = column j of B
    return gemm(M, N, K, ahat, K, False, bhat_t, K, True, alpha, beta, cin,
                N if cin is not None else None, rows)


def gemm_dense(A, B, alpha=1.0, beta=0.0, Cin=None, rows=None):
    """Convenience form on logical float64 matrices A (M x K), B (K x N)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    return gemm(M, N, K, A, K, False, B, N, False, alpha, beta,
                None if Cin is None else np.asarray(Cin, dtype=np.float64),
                N, rows)


def epilogue(c, bias=None, activation="none"):
    """Fused linear-layer epilogue applied to a product C (beyond the
    report, whose GEMM is the bare product; the layer is the deep-learning
    use its Introduction names): act(C[i][j] + bias[j]) in FP64, bias one
    value per output column.  Activations by their definitions:
    relu max(v, 0) (NaN passes through), gelu v * Phi(v) with
    Phi(v) = (1 + erf(v / sqrt 2)) / 2 the standard normal distribution,
    silu v * sigma(v) with sigma(v) = 1 / (1 + exp(-v))."""
    from scipy import special
    v = np.array(c, dtype=np.float64, copy=True)
    if bias is not None:
        v = v + np.asarray(bias, dtype=np.float64)[None, :]
    if activation == "none":
        return v
    if activation == "relu":
        return np.where(v < 0, 0.0, v)
    if activation == "gelu":
        return v * 0.5 * (1.0 + special.erf(v / np.sqrt(2.0)))
    if activation == "silu":
        return v * special.expit(v)
    raise ValueError(activation)


def rel_frobenius(x, ref) -> float:
    """||x - ref||_F / ||ref||_F (absolute error when ||ref||_F == 0)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = float(np.linalg.norm((x - ref).ravel()))
    den = float(np.linalg.norm(ref.ravel()))
    return num / den if den > 0 else num
