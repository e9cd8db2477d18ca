"""Shared helpers of the GPU parity tests: build seeded inputs, run the HIP
path through the C ABI, and compute the oracle on the same rounded inputs."""
import numpy as np
import pytest
import torch

import paper_2407_00044_amd as sk
from oracle import gemm as og
from paper_2407_00044_amd import synth

gpu = pytest.mark.gpu

TOL = {"f32": 1e-5, "f16": 1e-4, "bf16": 1e-4, "e4m3": 1e-4}
ELEM = {"f32": 4, "f16": 2, "bf16": 2, "e4m3": 1}
OUT_TORCH = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def dev():
    return torch.device("cuda", 0)


def x64_to_e4m3(x64):
    return torch.from_numpy(np.ascontiguousarray(x64)).to(torch.float8_e4m3fn)


class Operand:
    """A seeded operand: rounded CPU tensor, its GPU placement and codes."""

    def __init__(self, x64, dtype, col_major, ld=None, pad_align=True, scaled=True,
                 pad_nan=False):
        self.dtype = dtype
        self.col_major = col_major
        if dtype == "e4m3" and scaled:
            self.t, self.scale = synth.fp8_scaled(x64)
        elif dtype == "e4m3":
            # small integers are exact e4m3 values: no per-tensor scaling
            self.t, self.scale = x64_to_e4m3(x64), 1.0
        else:
            self.t, self.scale = synth.round_to(x64, dtype), 1.0
        rows, cols = x64.shape
        inner = rows if col_major else cols
        if ld is None and pad_align:
            ld = synth.ld_aligned(inner, ELEM[dtype])
        self.view, store, self.ld = synth.place(self.t, col_major, ld, device=dev())
        self.codes = synth.codes(store.cpu())
        if pad_nan and self.ld > inner:
            # row padding (never part of the product) holds NaN on the GPU
            if dtype == "e4m3":
                store.view(torch.uint8)[:, inner:] = 0x7F
            else:
                store[:, inner:] = float("nan")
        self.x64 = x64

    def decoded(self):
        """Storage decoded exactly to float64 (oracle input)."""
        return og.decode(self.dtype, self.codes)


def make_inputs(M, N, K, dtype, a_col=False, b_col=True, seed=1, dist="uniform", lda=None,
                ldb=None, pad_nan=False):
    if dist == "uniform":
        a64 = synth.uniform((M, K), seed)
        b64 = synth.uniform((K, N), seed + 1000)
    elif dist == "normal":
        a64 = synth.normal((M, K), seed)
        b64 = synth.normal((K, N), seed + 1000)
    elif dist == "int":
        a64 = synth.integers((M, K), seed)
        b64 = synth.integers((K, N), seed + 1000)
    else:
        raise ValueError(dist)
    scaled = dist != "int"
    return (Operand(a64, dtype, a_col, lda, scaled=scaled, pad_nan=pad_nan),
            Operand(b64, dtype, b_col, ldb, scaled=scaled, pad_nan=pad_nan))


def oracle(A, B, M, N, K, alpha=1.0, beta=0.0, cin=None, rows=None):
    s = alpha * A.scale * B.scale
    return og.gemm(M, N, K, A.decoded(), A.ld, A.col_major, B.decoded(), B.ld, B.col_major,
                   s, beta, cin, N if cin is not None else None, rows)


def oracle_unrounded(A, B, alpha=1.0, beta=0.0, cin=None, rows=None):
    """Same product on the float64 draws before rounding (reported only)."""
    return og.gemm_dense(A.x64, B.x64, alpha, beta, cin, rows)


def run(A, B, cfg, out_dtype="f32", alpha=1.0, beta=0.0, C=None):
    out = sk.gemm(A.view, B.view, C, alpha=alpha, beta=beta, out_dtype=OUT_TORCH[out_dtype],
                  scale_a=A.scale, scale_b=B.scale, config=cfg)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    return out


def as64(t):
    return t.float().cpu().numpy().astype(np.float64)


def rel_err(x, ref):
    return og.rel_frobenius(x, ref)
