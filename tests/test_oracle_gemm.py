"""Pins of the FP64 oracle GEMM and its exact decoders (CPU only).

Every check here compares the oracle with something other than itself:
exact algebraic identities, integer arithmetic done by numpy in int64, a
float64 library matmul, or torch's own format conversions.  Each plausible
slip in the oracle (a transposed operand, a wrong leading dimension, a
dropped alpha/beta term, a wrong exponent bias) fails at least one test.
"""
import numpy as np
import pytest
import torch

from oracle import gemm as og


def _store(X, col_major, ld_pad=0):
    """Storage array + leading dimension of logical matrix X (rows x cols)."""
    X = np.asarray(X, dtype=np.float64)
    if col_major:
        X = X.T
    r, c = X.shape
    ld = c + ld_pad
    buf = np.full((r, ld), np.nan)
    buf[:, :c] = X
    return buf, ld


def _run(A, B, a_col, b_col, alpha=1.0, beta=0.0, Cin=None, pad=0, rows=None):
    M, K = A.shape
    _, N = B.shape
    a, lda = _store(A, a_col, pad)
    b, ldb = _store(B, b_col, pad)
    return og.gemm(M, N, K, a, lda, a_col, b, ldb, b_col, alpha, beta, Cin,
                   N if Cin is not None else None, rows)


LAYOUTS = [(False, False), (False, True), (True, False), (True, True)]


@pytest.mark.parametrize("a_col,b_col", LAYOUTS)
def test_identity_gives_B_exactly(oracle_built, a_col, b_col):
    rng = np.random.default_rng(0)
    n, N = 37, 53
    B = rng.uniform(-1, 1, (n, N))
    C = _run(np.eye(n), B, a_col, b_col, alpha=1.0, pad=3)
    assert np.array_equal(C, B)
    C2 = _run(np.eye(n), B, a_col, b_col, alpha=-2.5)
    assert np.array_equal(C2, -2.5 * B)


@pytest.mark.parametrize("a_col,b_col", LAYOUTS)
def test_integer_products_exact(oracle_built, a_col, b_col):
    # Non-square, non-symmetric integer operands: a transposed operand or a
    # wrong stride cannot reproduce numpy's exact int64 product.
    rng = np.random.default_rng(1)
    M, N, K = 29, 41, 67
    A = rng.integers(-4, 5, (M, K))
    B = rng.integers(-4, 5, (K, N))
    ref = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    C = _run(A, B, a_col, b_col, pad=5)
    assert np.array_equal(C, ref)


def test_rank1_exact(oracle_built):
    rng = np.random.default_rng(2)
    M, N, K = 31, 17, 23
    u = rng.integers(-8, 9, M).astype(np.float64)
    v = rng.integers(-8, 9, K).astype(np.float64)
    B = rng.integers(-8, 9, (K, N)).astype(np.float64)
    A = np.outer(u, v)
    ref = np.outer(u, v @ B)          # C = u (v^T B), all exact integers
    assert np.array_equal(_run(A, B, False, True), ref)


def test_alpha_beta_terms(oracle_built):
    rng = np.random.default_rng(3)
    M, N, K = 16, 24, 8
    A = rng.integers(-3, 4, (M, K)).astype(np.float64)
    B = rng.integers(-3, 4, (K, N)).astype(np.float64)
    Cin = rng.integers(-3, 4, (M, N)).astype(np.float64)
    AB = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    # alpha, beta powers of two keep everything exact
    C = _run(A, B, False, False, alpha=0.5, beta=-2.0, Cin=Cin)
    assert np.array_equal(C, 0.5 * AB - 2.0 * Cin)
    # beta == 0 never reads Cin, even when Cin holds NaN
    C = _run(A, B, False, False, alpha=1.0, beta=0.0,
             Cin=np.full((M, N), np.nan))
    assert np.array_equal(C, AB)
    # A == 0 leaves exactly beta * Cin
    C = _run(np.zeros((M, K)), B, False, False, alpha=3.0, beta=0.25, Cin=Cin)
    assert np.array_equal(C, 0.25 * Cin)


def test_k_zero_is_beta_c(oracle_built):
    Cin = np.arange(12, dtype=np.float64).reshape(3, 4)
    C = og.gemm(3, 4, 0, np.zeros(0), 1, False, np.zeros(0), 4, False,
                1.0, 0.5, Cin, 4)
    assert np.array_equal(C, 0.5 * Cin)


@pytest.mark.parametrize("a_col,b_col", LAYOUTS)
def test_matches_numpy_float64(oracle_built, a_col, b_col):
    rng = np.random.default_rng(4)
    M, N, K = 96, 80, 512
    A = rng.uniform(-1, 1, (M, K))
    B = rng.uniform(-1, 1, (K, N))
    C = _run(A, B, a_col, b_col)
    assert og.rel_frobenius(C, A @ B) < 1e-13


def test_row_sample_equals_full(oracle_built):
    rng = np.random.default_rng(5)
    M, N, K = 50, 33, 40
    A = rng.uniform(-1, 1, (M, K))
    B = rng.uniform(-1, 1, (K, N))
    Cin = rng.uniform(-1, 1, (M, N))
    full = _run(A, B, True, False, alpha=1.5, beta=0.5, Cin=Cin)
    rows = [49, 0, 7, 7, 22]
    part = _run(A, B, True, False, alpha=1.5, beta=0.5, Cin=Cin, rows=rows)
    assert np.array_equal(part, full[rows])


def test_row_sample_rejects_bad_rows(oracle_built):
    A = np.ones((4, 4))
    with pytest.raises(ValueError):
        _run(A, A, False, False, rows=[4])


def _exhaustive(codes, view_dtype, torch_dtype, decoder):
    ref = torch.from_numpy(codes.view(view_dtype)).view(torch_dtype).to(
        torch.float64).numpy()
    got = decoder(codes)
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(got))
    assert np.array_equal(ref[~nan], got[~nan])
    assert np.array_equal(np.signbit(ref[~nan]), np.signbit(got[~nan]))


def test_decode_bf16_all_codes():
    _exhaustive(np.arange(1 << 16, dtype=np.uint16), np.int16, torch.bfloat16,
                og.decode_bf16)


def test_decode_f16_all_codes():
    _exhaustive(np.arange(1 << 16, dtype=np.uint16), np.int16, torch.float16,
                og.decode_f16)


def test_decode_e4m3fn_all_codes():
    codes = np.arange(256, dtype=np.uint8)
    _exhaustive(codes, np.uint8, torch.float8_e4m3fn, og.decode_e4m3fn)
    vals = og.decode_e4m3fn(codes)
    assert np.nanmax(vals) == 448.0 and np.isnan(vals).sum() == 2


def test_decode_e5m2_all_codes():
    # against torch's e5m2, then the published extremes of the OCP format,
    # then the identity with the upper byte of an IEEE binary16 code
    codes = np.arange(256, dtype=np.uint8)
    _exhaustive(codes, np.uint8, torch.float8_e5m2, og.decode_e5m2)
    vals = og.decode_e5m2(codes)
    assert vals[0x7B] == 57344.0 and np.nanmax(vals[np.isfinite(vals)]) == 57344.0
    assert vals[0x04] == 2.0 ** -14 and vals[0x01] == 2.0 ** -16 and vals[0x03] == 0.75 * 2 ** -14
    assert vals[0x7C] == np.inf and vals[0xFC] == -np.inf and np.isnan(vals).sum() == 6
    assert vals[0x3C] == 1.0 and vals[0xC0] == -2.0 and vals[0x80] == 0 and np.signbit(vals[0x80])
    f16 = og.decode_f16(codes.astype(np.uint16) << 8)
    assert np.array_equal(np.isnan(f16), np.isnan(vals))
    assert np.array_equal(f16[~np.isnan(f16)], vals[~np.isnan(vals)])


def test_mx_operand_e5m2_scales_exactly():
    # a block of e5m2 codes times 2^(s - 127), s per 32 elements
    rng = np.random.default_rng(12)
    c = rng.integers(0, 256, size=(3, 64), dtype=np.uint8)
    c[(c & 0x7C) == 0x7C] = 0x3C             # no infinities or NaN in this pin
    s = np.array([[120, 130], [127, 127], [0, 254]], dtype=np.uint8)
    got = og.mx_operand(c.reshape(-1), 64, s.reshape(-1), 2, 3, 64, elem="e5m2")
    want = og.decode_e5m2(c) * np.repeat(np.ldexp(1.0, s.astype(int) - 127), 32, axis=1)
    assert np.array_equal(got, want)


def test_decode_f32_roundtrip():
    rng = np.random.default_rng(6)
    x = rng.standard_normal(1000).astype(np.float32)
    assert np.array_equal(og.decode_f32(x.view(np.uint32)), x.astype(np.float64))


def test_rel_frobenius_basics():
    assert og.rel_frobenius([3.0, 4.0], [3.0, 4.0]) == 0.0
    assert og.rel_frobenius([3.0, 4.0], [0.0, 0.0]) == 5.0
    assert abs(og.rel_frobenius([3.0, 5.0], [3.0, 4.0]) - 0.2) < 1e-15


# ---------------------------------------------------------------------------
# MXFP8 (OCP MX block scaling).

def test_decode_e8m0_all_codes():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e8m0fnu).to(torch.float64).numpy()
    got = og.decode_e8m0(codes)
    assert np.array_equal(got, ref, equal_nan=True)
    # the format itself: 2^(e-127), e = 255 NaN
    assert got[127] == 1.0 and got[128] == 2.0 and got[0] == 2.0 ** -127
    assert np.isnan(got[255]) and not np.isnan(got[:255]).any()


def _mx_case(M, N, K, seed, ldpad=0, spad=0):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 256, size=(M, K + ldpad)).astype(np.uint8)
    b = rng.integers(0, 256, size=(N, K + ldpad)).astype(np.uint8)
    a[(a & 0x7F) == 0x7F] = 0x10            # no NaN codes
    b[(b & 0x7F) == 0x7F] = 0x10
    sa = rng.integers(120, 135, size=(M, K // 32 + spad)).astype(np.uint8)
    sb = rng.integers(120, 135, size=(N, K // 32 + spad)).astype(np.uint8)
    return a, b, sa, sb


def test_mx_unit_scales_equal_plain_e4m3_product(oracle_built):
    M, N, K = 7, 5, 96
    a, b, _, _ = _mx_case(M, N, K, 1, ldpad=3)
    one_a = np.full((M, K // 32), 127, np.uint8)
    one_b = np.full((N, K // 32), 127, np.uint8)
    got = og.gemm_mx(M, N, K, a, K + 3, one_a, K // 32, b, K + 3, one_b, K // 32)
    plain = og.gemm(M, N, K, og.decode_e4m3fn(a.reshape(-1)), K + 3, False,
                    og.decode_e4m3fn(b.reshape(-1)), K + 3, True)
    assert np.array_equal(got, plain)


def test_mx_brute_force_exact_rationals(oracle_built):
    # every block-scaled element is a dyadic rational: the exact sum (with
    # Fractions) rounded once to float64 agrees with the FP64 loop to its
    # summation error
    from fractions import Fraction
    M, N, K = 3, 4, 64
    a, b, sa, sb = _mx_case(M, N, K, 2, ldpad=0, spad=2)
    lds = K // 32 + 2
    got = og.gemm_mx(M, N, K, a, K, sa, lds, b, K, sb, lds)
    ea = og.decode_e4m3fn(a.reshape(-1))
    eb = og.decode_e4m3fn(b.reshape(-1))
    for i in range(M):
        for j in range(N):
            acc = Fraction(0)
            for k in range(K):
                fa = Fraction(ea[i * K + k]) * Fraction(2) ** (int(sa[i, k // 32]) - 127)
                fb = Fraction(eb[j * K + k]) * Fraction(2) ** (int(sb[j, k // 32]) - 127)
                acc += fa * fb
            assert abs(got[i, j] - float(acc)) <= 1e-13 * max(1.0, abs(float(acc)))


def test_mx_block_scale_moves_one_block_by_a_power_of_two(oracle_built):
    # raising the scale code of one block of one row of A by d multiplies
    # that block's contribution to the row of C by 2^d and nothing else
    M, N, K = 4, 6, 128
    a, b, sa, sb = _mx_case(M, N, K, 3)
    base = og.gemm_mx(M, N, K, a, K, sa, K // 32, b, K, sb, K // 32)
    sa2 = sa.copy()
    sa2[2, 1] += 3
    bumped = og.gemm_mx(M, N, K, a, K, sa2, K // 32, b, K, sb, K // 32)
    # the block's own contribution, by the oracle on that block alone
    mask = np.zeros((M, K), np.uint8)
    a_blk = np.where(np.arange(K)[None, :] // 32 == 1, a, 0).astype(np.uint8)
    part = og.gemm_mx(M, N, K, a_blk, K, sa, K // 32, b, K, sb, K // 32)
    expect = base.copy()
    expect[2] += (2.0 ** 3 - 1.0) * part[2]
    assert np.allclose(bumped, expect, rtol=1e-13, atol=0)
    assert np.array_equal(np.delete(bumped, 2, axis=0), np.delete(base, 2, axis=0))
    del mask


def test_mx_quantize_round_trip_within_e4m3_precision():
    from paper_2407_00044_amd import synth
    x = np.random.default_rng(4).standard_normal((5, 256)) * np.logspace(-3, 3, 256)[None, :]
    q, s = synth.mx_quantize(x)
    assert q.dtype == torch.float8_e4m3fn and s.shape == (5, 8)
    back = og.mx_operand(synth.codes(q), 256, s, 8, 5, 256)
    rel = np.abs(back - x) / np.maximum(np.abs(x), 1e-300)
    # e4m3 keeps 3 fraction bits: relative rounding error <= 2^-4 for values
    # in each block's normal range; the block's smallest values may be
    # subnormal, so check the error against the block's largest value too
    blk_max = np.repeat(np.abs(x).reshape(5, 8, 32).max(axis=2), 32, axis=1)
    assert np.all((rel <= 2.0 ** -4) | (np.abs(back - x) <= blk_max * 2.0 ** -9))


# ---------------------------------------------------------------------------
# Fused epilogue: bias per output column, then an activation.

def test_epilogue_bias_is_per_column_on_a_rank_one_product(oracle_built):
    # C = u v^T + bias[j] on a non-square shape: a bias broadcast along the
    # wrong axis, or dropped, fails (values exact in FP64)
    u = np.arange(1, 6, dtype=np.float64)            # M = 5
    v = np.arange(-3, 4, dtype=np.float64)           # N = 7
    bias = np.array([0.5, -1, 2, 0, 8, -0.25, 3])
    c = og.epilogue(og.gemm_dense(u[:, None], v[None, :]), bias)
    assert np.array_equal(c, np.outer(u, v) + bias[None, :])
    assert np.array_equal(og.epilogue(c), c)          # "none" is the identity


def test_epilogue_relu_hand_values():
    x = np.array([[-2.0, -0.0, 0.0, 1.5, np.inf, -np.inf, np.nan]])
    r = og.epilogue(x, activation="relu")
    assert np.array_equal(r[0, :6], [0, 0, 0, 1.5, np.inf, 0])
    assert np.isnan(r[0, 6])


def test_epilogue_gelu_normal_quantile_and_odd_part():
    # Phi(1.959963984540054) = 0.975 (the 97.5% point of the standard
    # normal), so GELU(z) = 0.975 z there; Phi(0) = 1/2; and since erf is odd,
    # GELU(x) - GELU(-x) = x for every x
    z = 1.959963984540054
    g = og.epilogue(np.array([[z, -z, 0.0, 1.0]]), activation="gelu")[0]
    assert abs(g[0] - 0.975 * z) <= 1e-14 * z
    assert abs(g[1] + 0.025 * z) <= 1e-13 * z
    assert g[2] == 0.0
    x = np.random.default_rng(7).normal(scale=3, size=(4, 50))
    d = og.epilogue(x, activation="gelu") - og.epilogue(-x, activation="gelu")
    assert np.max(np.abs(d - x)) <= 1e-14 * np.max(np.abs(x))
    # far tails: GELU -> x for large x, -> 0 for very negative x
    t = og.epilogue(np.array([[40.0, -40.0]]), activation="gelu")[0]
    assert t[0] == 40.0 and abs(t[1]) < 1e-300


def test_epilogue_silu_closed_forms():
    # sigma(ln 3) = 3/4, so SiLU(ln 3) = (3/4) ln 3; sigma(x) + sigma(-x) = 1
    # gives SiLU(x) - SiLU(-x) = x; huge negative inputs give 0, not NaN
    s = og.epilogue(np.array([[np.log(3.0), 0.0, -800.0, 800.0]]), activation="silu")[0]
    assert abs(s[0] - 0.75 * np.log(3.0)) <= 1e-15
    assert s[1] == 0.0 and s[2] == 0.0 and s[3] == 800.0
    x = np.random.default_rng(8).normal(scale=4, size=(3, 40))
    d = og.epilogue(x, activation="silu") - og.epilogue(-x, activation="silu")
    assert np.max(np.abs(d - x)) <= 1e-14 * np.max(np.abs(x))


def test_epilogue_bias_before_activation():
    # act(c + b), not act(c) + b: with c = -1 and b = 2, relu gives 1 (the
    # other order would give 2)
    r = og.epilogue(np.full((2, 3), -1.0), np.full(3, 2.0), "relu")
    assert np.array_equal(r, np.ones((2, 3)))


# ---------------------------------------------------------------------------
# MXFP4: OCP FP4 (E2M1) elements, two per byte, with E8M0 block scales.

def test_decode_e2m1_all_codes():
    # the OCP MX format's E2M1 table: magnitudes 0, 0.5, 1, 1.5, 2, 3, 4, 6 for
    # codes 0..7, the same negated for 8..15 (sign bit 3)
    table = [0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0]
    got = og.decode_e2m1(np.arange(16))
    assert np.array_equal(got[:8], table)
    assert np.array_equal(got[8:], [-v for v in table])
    assert np.signbit(got[8])                     # code 8 is -0
    # only the low nibble of a wider integer is a code
    assert np.array_equal(og.decode_e2m1(np.arange(16) + 0x30), got)


def test_unpack_fp4_low_nibble_first():
    codes = og.unpack_fp4(np.array([0x21, 0xF7, 0x0A], dtype=np.uint8), 5)
    assert list(codes) == [0x1, 0x2, 0x7, 0xF, 0xA]


def test_mx_fp4_product_brute_force_exact_rationals(oracle_built):
    # an independent evaluation: exact rational arithmetic over the decoded
    # table, the scales applied per block of 32 K-values
    from fractions import Fraction
    rng = np.random.default_rng(11)
    M, N, K = 3, 2, 64
    a = rng.integers(0, 256, size=(M, K // 2)).astype(np.uint8)
    b = rng.integers(0, 256, size=(N, K // 2)).astype(np.uint8)
    sa = rng.integers(120, 135, size=(M, K // 32)).astype(np.uint8)
    sb = rng.integers(120, 135, size=(N, K // 32)).astype(np.uint8)
    table = [Fraction(v) for v in (0, 0.5, 1, 1.5, 2, 3, 4, 6)]

    def val(byte_row, k):
        code = (int(byte_row[k // 2]) >> (4 * (k % 2))) & 15
        v = table[code & 7]
        return -v if code & 8 else v

    def scale(e):
        return Fraction(2) ** (int(e) - 127)
    got = og.gemm_mx(M, N, K, a, K, sa, K // 32, b, K, sb, K // 32, elem="e2m1")
    for i in range(M):
        for j in range(N):
            exact = sum(val(a[i], k) * scale(sa[i, k // 32]) * val(b[j], k) * scale(sb[j, k // 32])
                        for k in range(K))
            assert got[i, j] == float(exact)


def test_mx_fp4_unit_scales_equal_the_plain_product(oracle_built):
    rng = np.random.default_rng(12)
    M, N, K = 5, 4, 96
    a = rng.integers(0, 256, size=(M, K // 2)).astype(np.uint8)
    b = rng.integers(0, 256, size=(N, K // 2)).astype(np.uint8)
    ones_a = np.full((M, K // 32), 127, np.uint8)
    ones_b = np.full((N, K // 32), 127, np.uint8)
    A = og.decode_e2m1(og.unpack_fp4(a, M * K)).reshape(M, K)
    B = og.decode_e2m1(og.unpack_fp4(b, N * K)).reshape(N, K).T
    got = og.gemm_mx(M, N, K, a, K, ones_a, K // 32, b, K, ones_b, K // 32, elem="e2m1")
    assert np.array_equal(got, A @ B)            # small integers and halves: exact


def test_mx4_quantize_round_trip_within_e2m1_precision():
    # every element within half the E2M1 spacing at its magnitude (0.5 below
    # 2, 1 below 4, 2 up to 6, times the block's power of two); values on
    # the grid come back exactly; the block maximum never saturates
    from paper_2407_00044_amd import synth
    x = np.random.default_rng(5).standard_normal((5, 256)) * np.logspace(-3, 3, 256)[None, :]
    p, s = synth.mx4_quantize(x)
    assert p.dtype == np.uint8 and p.shape == (5, 128) and s.shape == (5, 8)
    back = og.mx_operand(p, 256, s, 8, 5, 256, elem="e2m1")
    scale = np.repeat(og.decode_e8m0(s), 32, axis=1)
    y = np.abs(x) / scale                              # in [0, 6] by the choice of X
    assert np.all(y <= 6.0)
    half_spacing = np.where(y < 2, 0.25, np.where(y < 4, 0.5, 1.0)) * scale
    assert np.all(np.abs(back - x) <= half_spacing)
    grid = np.array([[0.5, -1.5, 3.0, 6.0] * 8])          # one block on the grid, scale 2^0
    pg, sg = synth.mx4_quantize(grid)
    assert sg[0, 0] == 127
    assert np.array_equal(og.mx_operand(pg, 32, sg, 1, 1, 32, elem="e2m1"), grid)


# ---------------------------------------------------------------------------
# MXFP6 (OCP FP6 E2M3 and E3M2 elements)

def test_fp6_decoders_against_the_format_tables():
    # the OCP MX formats' published extremes: E2M3 max normal 7.5, min
    # normal 1.0, max subnormal 0.875, min subnormal 0.125; E3M2 28.0, 0.25,
    # 0.1875, 0.0625; 32 distinct increasing magnitudes, sign bit 5
    for dec, ext in [(og.decode_e2m3, (7.5, 1.0, 0.875, 0.125)),
                     (og.decode_e3m2, (28.0, 0.25, 0.1875, 0.0625))]:
        v = dec(np.arange(64))
        mag = v[:32]
        assert np.all(np.diff(mag) > 0) and mag[0] == 0.0
        assert np.array_equal(v[32:], -mag)
        normals = mag[mag >= ext[1]]
        subnormals = mag[(mag > 0) & (mag < ext[1])]
        assert (normals.max(), normals.min(), subnormals.max(), subnormals.min()) == ext
        # subnormals are evenly spaced by the smallest one
        assert np.allclose(np.diff(np.concatenate([[0.0], subnormals])), ext[3])


def test_fp6_unpack_bit_order_hand_worked():
    # codes 1, 2, 3, 4 at bits 0-5, 6-11, 12-17, 18-23:
    # 1 + 2*2^6 + 3*2^12 + 4*2^18 = 0x103081 -> bytes 0x81 0x30 0x10
    assert list(og.unpack_fp6(np.array([0x81, 0x30, 0x10]), 4)) == [1, 2, 3, 4]
    # the top code in every slot: all 24 bits set
    assert list(og.unpack_fp6(np.array([0xFF, 0xFF, 0xFF]), 4)) == [63] * 4


def test_fp6_pack_round_trip_and_quantizer():
    from paper_2407_00044_amd import synth
    rng = np.random.default_rng(7)
    c = rng.integers(0, 64, size=(5, 96))
    packed = synth.pack_fp6(c)
    assert packed.shape == (5, 72)
    for r in range(5):
        assert np.array_equal(og.unpack_fp6(packed[r], 96), c[r])
    for fmt, dec in (("e2m3", og.decode_e2m3), ("e3m2", og.decode_e3m2)):
        grid = dec(np.arange(64))
        # every representable value is its own rounding
        assert np.array_equal(dec(synth.fp6_rne(grid, fmt)), grid)
        # the midpoint of two neighbours goes to the even code; beyond the
        # largest value saturates
        mag = grid[:32]
        mids = (mag[:-1] + mag[1:]) / 2
        got = synth.fp6_rne(mids, fmt)
        assert np.all(got % 2 == 0)
        assert dec(synth.fp6_rne(np.array([1e9, -1e9]), fmt)).tolist() == [mag[-1], -mag[-1]]
    # MX quantisation: the block's largest magnitude lands in the top binade
    x = synth.normal((4, 128), 8)
    packed, sc = synth.mx6_quantize(x, "e2m3")
    vals = og.decode_e2m3(og.unpack_fp6(packed.reshape(-1), 4 * 128)).reshape(4, 128)
    for b in range(4):
        blk = np.abs(x[:, 32 * b:32 * b + 32]).max(axis=1) / np.ldexp(1.0, sc[:, b].astype(int) - 127)
        assert np.all((blk <= 7.5) & (blk > 7.5 / 2))
    assert np.max(np.abs(vals)) <= 7.5
