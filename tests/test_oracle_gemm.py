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


def test_decode_f32_roundtrip():
    rng = np.random.default_rng(6)
    x = rng.standard_normal(1000).astype(np.float32)
    assert np.array_equal(og.decode_f32(x.view(np.uint32)), x.astype(np.float64))


def test_rel_frobenius_basics():
    assert og.rel_frobenius([3.0, 4.0], [3.0, 4.0]) == 0.0
    assert og.rel_frobenius([3.0, 4.0], [0.0, 0.0]) == 5.0
    assert abs(og.rel_frobenius([3.0, 5.0], [3.0, 4.0]) - 0.2) < 1e-15
