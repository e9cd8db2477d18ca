"""Stream-K GEMM for AMD MI355X (gfx950).

C = alpha * A @ B + beta * C computed by hand-written HIP kernels with
Stream-K's work-centric decomposition: the MAC-loop iterations of all output
tiles are split evenly over one persistent workgroup per compute unit, and
tiles that straddle workgroups are finished by a partial-sum fixup.

The compute path is libstreamk.so (C ABI in include/streamk.h); this package
is its Python binding.  Importing it does not load the library; the first
call does, and fails loudly if the library has not been built.
"""
from ._abi import LIB_PATH, StreamKError, load  # noqa: F401
from . import tune  # noqa: F401
from .api import (ACTIVATIONS, Config, GroupedGemm, StreamKLinearFn, Workspace,  # noqa: F401
                  check_device_error, check_noalloc_error, cost_model, default_tile, device_query,
                  gemm, gemm_debug, gemm_mx, gemm_mx4, gemm_mx6, gemm_noalloc, k_contiguous,
                  launch_params, linear, pack_pays, plan, plan_order, schedule,
                  supported_tiles, transpose)
