"""ctypes mirror of include/streamk.h (argument marshalling only).

Every step of a GEMM runs in libstreamk.so; this module only declares the C
structures and prototypes and loads the library.  A missing library is an
error -- there is no fallback path.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstreamk.so")

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_f32 = ctypes.c_float
c_vp = ctypes.c_void_p

# status codes
SK_OK = 0
SK_ERR_INVALID_ARG = -1
SK_ERR_UNSUPPORTED = -2
SK_ERR_WORKSPACE = -3
SK_ERR_OCCUPANCY = -4
SK_ERR_HIP = -5
SK_ERR_CAPACITY = -6
SK_ERR_DEVICE_TIMEOUT = -7

# dtypes / layouts / modes / roles
SK_F32, SK_F16, SK_BF16, SK_F8E4M3, SK_MXF8E4M3, SK_MXF4E2M1 = 0, 1, 2, 3, 4, 5
SK_MXF6E2M3, SK_MXF6E3M2, SK_MXF8E5M2, SK_F8E5M2 = 6, 7, 8, 9
SK_ROW_MAJOR, SK_COL_MAJOR = 0, 1
SK_MODE_HYBRID, SK_MODE_SK, SK_MODE_DP, SK_MODE_AUTO = 0, 1, 2, 3
SK_ROLE_FULL, SK_ROLE_FINISH, SK_ROLE_PARTIAL, SK_ROLE_DP = 0, 1, 2, 3
SK_ACT_NONE, SK_ACT_RELU, SK_ACT_GELU, SK_ACT_SILU = 0, 1, 2, 3

MODES = {"hybrid": SK_MODE_HYBRID, "sk": SK_MODE_SK, "dp": SK_MODE_DP, "auto": SK_MODE_AUTO}


class SkProblem(ctypes.Structure):
    _fields_ = [("M", c_i64), ("N", c_i64), ("K", c_i64),
                ("layout_a", c_i32), ("layout_b", c_i32),
                ("lda", c_i64), ("ldb", c_i64), ("ldc", c_i64),
                ("dtype_ab", c_i32), ("dtype_c", c_i32),
                ("alpha", c_f32), ("beta", c_f32),
                ("scale_a", c_f32), ("scale_b", c_f32),
                ("bias", ctypes.c_void_p), ("activation", c_i32), ("reserved", c_i32)]


class SkConfig(ctypes.Structure):
    _fields_ = [("block_m", c_i32), ("block_n", c_i32), ("block_k", c_i32),
                ("num_cu", c_i32), ("wg_per_cu", c_i32), ("mode", c_i32),
                ("dp_tiles", c_i64), ("group_m", c_i32), ("xcd_remap", c_i32),
                ("spin_limit", c_i64), ("min_iters", c_i32)]


class SkSegment(ctypes.Structure):
    _fields_ = [("wg", c_i32), ("problem", c_i32), ("tile", c_i32),
                ("tile_m", c_i32), ("tile_n", c_i32),
                ("k_begin", c_i32), ("k_end", c_i32),
                ("role", c_i32), ("npeers", c_i32)]


class SkPlanInfo(ctypes.Structure):
    _fields_ = [("T", c_i64), ("S", c_i64), ("W", c_i64), ("g", c_i64),
                ("q", c_i64), ("rho", c_i64), ("workspace_bytes", c_i64),
                ("max_iters", c_i64), ("group_m", c_i64), ("dp_grid", c_i64),
                ("predicted_us", ctypes.c_double), ("predicted_dp_us", ctypes.c_double)]


class SkDebug(ctypes.Structure):
    _fields_ = [("trace", c_vp), ("trace_capacity", c_i64),
                ("trace_count", c_vp), ("cover", c_vp),
                ("cover_stride", c_i64), ("partial_delay", c_i32),
                ("reverse_ids", c_i32)]


class SkGroupedPlan(ctypes.Structure):
    _fields_ = [("nprobs", c_i32), ("mode", c_i32),
                ("dtype_ab", c_i32), ("dtype_c", c_i32),
                ("layout_a", c_i32), ("layout_b", c_i32),
                ("block_m", c_i32), ("block_n", c_i32), ("block_k", c_i32),
                ("T", c_i64), ("S", c_i64), ("W", c_i64), ("g", c_i64),
                ("q", c_i64), ("rho", c_i64), ("workspace_bytes", c_i64),
                ("xcd_remap", c_i32), ("group_m", c_i32),
                ("spin_limit", c_i64), ("all_aligned", c_i32), ("max_iters", c_i64)]


P = ctypes.POINTER

# name -> (restype, argtypes); every entry point returns sk_status except
# sk_status_string.
PROTOTYPES = {
    "sk_status_string": (ctypes.c_char_p, [c_i32]),
    "sk_device_query": (c_i32, [P(c_i32), P(c_i32), P(SkConfig), c_i32]),
    "sk_supported_tiles": (c_i32, [c_i32, P(c_i32), c_i32, P(c_i32)]),
    "sk_plan": (c_i32, [P(SkProblem), c_i32, P(SkConfig), P(SkPlanInfo)]),
    "sk_plan_order": (c_i32, [P(SkProblem), c_i32, P(SkConfig), P(c_i32)]),
    "sk_cost_model": (c_i32, [c_i32, c_i32, c_i32, P(ctypes.c_float), c_i32]),
    "sk_schedule": (c_i32, [P(SkProblem), c_i32, P(SkConfig), P(SkSegment), c_i64,
                            P(c_i64)]),
    "sk_workspace_size": (c_i32, [P(SkProblem), c_i32, P(SkConfig), P(ctypes.c_size_t)]),
    "sk_workspace_init": (c_i32, [c_vp, ctypes.c_size_t, c_vp]),
    "sk_gemm": (c_i32, [P(SkProblem), c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t,
                        P(SkConfig), c_vp]),
    "sk_gemm_mx": (c_i32, [P(SkProblem), c_vp, c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp,
                           c_vp, ctypes.c_size_t, P(SkConfig), c_vp]),
    "sk_gemm_debug": (c_i32, [P(SkProblem), c_vp, c_vp, c_vp, c_vp, c_vp,
                              ctypes.c_size_t, P(SkConfig), P(SkDebug), c_vp]),
    "sk_check_device_error": (c_i32, [c_vp, ctypes.c_size_t, P(c_i32), c_vp]),
    "sk_gemm_noalloc": (c_i32, [P(SkProblem), c_vp, c_vp, c_vp, c_vp, P(SkConfig), c_vp]),
    "sk_grouped_desc_size": (c_i32, [c_i32, P(ctypes.c_size_t)]),
    "sk_grouped_prepare": (c_i32, [P(SkProblem), P(c_vp), P(c_vp), P(c_vp), P(c_vp),
                                   c_i32, P(SkConfig), c_vp, ctypes.c_size_t,
                                   P(SkGroupedPlan), c_vp]),
    "sk_grouped_prepare_mx": (c_i32, [P(SkProblem), P(c_vp), P(c_vp), P(c_vp), P(c_i64),
                                      P(c_vp), P(c_i64), P(c_vp), P(c_vp), c_i32, P(SkConfig),
                                      c_vp, ctypes.c_size_t, P(SkGroupedPlan), c_vp]),
    "sk_gemm_grouped": (c_i32, [P(SkGroupedPlan), c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "sk_gemm_grouped_debug": (c_i32, [P(SkGroupedPlan), c_vp, c_vp, ctypes.c_size_t,
                                      P(SkDebug), c_vp]),
    "sk_transpose": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_vp, c_i64, c_i32, c_vp]),
}

_lib = None


class StreamKError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        msg = status_string(status) if _lib is not None else str(status)
        super().__init__(f"{fn} failed: {msg} ({status})")


def load():
    """Load libstreamk.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; "
                "g.build()'` (hipcc --offload-arch=gfx950) first")
        # torch must own the HIP runtime before the library binds to it, so
        # that both share one runtime, one device context and the same streams.
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def status_string(status):
    return load().sk_status_string(status).decode()


def check(fn, status):
    if status != SK_OK:
        raise StreamKError(fn, status)
