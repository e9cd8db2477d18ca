"""Measurement conventions of the benchmark and reports.

The report's Table 1 (Results section) lists ms, TFLOP/s and GB/s per GEMM;
its TFLOP/s column is 2*M*N*K over the time and its GB/s column counts each
of A, B and C once at 2 bytes an element.  The arithmetic intensity it quotes
for 3840x4096x4096 (Methodology section) is that flop count over those
bytes.  MI355X peaks are the published dense figures at 2.4 GHz.
"""

PEAK_TFLOPS = {"f16": 2516.6, "bf16": 2516.6, "e4m3": 5033.2, "f32": 157.3}
HBM_GBS = 8000.0


def gemm_flops(M, N, K):
    """Multiply-adds of an M x N x K product, two flops each (beta*C and any
    padded or zero-filled work not counted)."""
    return 2.0 * M * N * K


def tflops(flops, ms):
    return flops / (ms * 1e-3) / 1e12


def operand_bytes(M, N, K, e_ab, e_c, beta_nonzero=False):
    """Algorithmic bytes of one GEMM: A and B read once, C written once (and
    read once more when beta != 0)."""
    return e_ab * (M * K + K * N) + e_c * M * N * (2 if beta_nonzero else 1)


def gbs(M, N, K, ms, e_ab=2, e_c=2):
    """Table 1's GB/s: operand bytes (A, B, C once each) per second, 1e9."""
    return operand_bytes(M, N, K, e_ab, e_c) / (ms * 1e-3) / 1e9


def arithmetic_intensity(M, N, K, e_ab=2, e_c=2):
    """Flops per operand byte."""
    return gemm_flops(M, N, K) / operand_bytes(M, N, K, e_ab, e_c)


def dp_efficiency(T, g):
    """Busy fraction of g cores running T equal tiles in waves of g."""
    return 1.0 if T == 0 else T / (-(-T // g) * g)


def roofline_time_s(M, N, K, e_ab, e_c, peak_tflops, beta_nonzero=False):
    """Lower bound on a GEMM's time: its flops at the matrix-core peak or its
    operand bytes at HBM bandwidth, whichever is longer."""
    return max(gemm_flops(M, N, K) / (peak_tflops * 1e12),
               operand_bytes(M, N, K, e_ab, e_c, beta_nonzero) / (HBM_GBS * 1e9))
