"""ctypes declarations of libqcemu.so (the C-ABI in include/qcemu.h).

Loading fails loudly when the library has not been built: there is no CPU
fallback for any entry point.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# QCE_LIB: another build of the same library (the host-sanitizer variant)
LIB_PATH = os.environ.get("QCE_LIB") or os.path.join(HERE, "libqcemu.so")

# qce_mode values
MODE_FP16X2, MODE_FP16X2_SCALED, MODE_BF16X3, MODE_FP32, MODE_AUTO = 0, 1, 2, 3, 4
MODE_NAMES = {MODE_FP16X2: "fp16x2", MODE_FP16X2_SCALED: "fp16x2_scaled",
              MODE_BF16X3: "bf16x3", MODE_FP32: "fp32", MODE_AUTO: "auto"}
MODE_BY_NAME = {v: k for k, v in MODE_NAMES.items()}
OPS = {"N": 0, "T": 1, "C": 2}
STATUS = {0: "QCE_SUCCESS", 1: "QCE_ERR_INVALID_VALUE", 2: "QCE_ERR_NOT_SUPPORTED",
          3: "QCE_ERR_ALLOC", 4: "QCE_ERR_HIP", 5: "QCE_ERR_INTERNAL"}

# every symbol include/qcemu.h declares
EXPORTS = (
    "qce_create", "qce_destroy", "qce_set_stream", "qce_set_mode", "qce_get_mode",
    "qce_set_underflow_tolerance", "qce_set_size_policy", "qce_get_size_policy", "qce_set_gemm_size_policy",
    "qce_set_gemm_tile",
    "qce_set_workspace",
    "qce_cgemm_workspace_size", "qce_cgemm_emulated", "qce_cgemm_emulated_noalloc",
    "qce_noalloc_scratch_bytes", "qce_get_last_decision",
    "qce_cgemm_batched_workspace_size", "qce_cgemm_strided_batched", "qce_cgemm_grouped",
    "qce_get_batch_decision",
    "qce_contract", "qce_group_begin", "qce_group_end", "qce_group_reset", "qce_permute", "qce_accumulate_f64", "qce_accumulate_n_f64", "qce_fidelity_f64",
    "qce_expstats", "qce_split", "qce_panel_bytes", "qce_split_panels", "qce_split_panels_bitmap",
    "qce_status_string", "qce_last_error",
    "qce_set_timing", "qce_set_timing_tag", "qce_reset_timing", "qce_get_timing",
)

PHASES = ("stats", "split", "gemm_fp16x2", "gemm_bf16x3", "gemm_fp32", "gemm_skipped",
          "permute", "other", "gemm_irregular", "gemm_batched")


class QceC32(ctypes.Structure):
    _fields_ = [("re", ctypes.c_float), ("im", ctypes.c_float)]


class QceGemmDesc(ctypes.Structure):
    _fields_ = [("opA", ctypes.c_int), ("opB", ctypes.c_int),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("alpha", QceC32), ("beta", QceC32),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64)]


class QceTensor(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("extents", ctypes.POINTER(ctypes.c_int64))]


class QceDecision(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("sA", ctypes.c_int32), ("sB", ctypes.c_int32),
                ("stats_taken", ctypes.c_int32),
                ("nnz", ctypes.c_int64 * 2), ("n1", ctypes.c_int64 * 2),
                ("n2", ctypes.c_int64 * 2), ("n3", ctypes.c_int64 * 2),
                ("nonfinite", ctypes.c_int64 * 2), ("emax", ctypes.c_int32 * 2)]


class QceTiming(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 10), ("count", ctypes.c_int64 * 10),
                ("gemms_by_mode", ctypes.c_int64 * 4)]


class QceError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


_lib = None


def load():
    """Load libqcemu.so; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2303_08989_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    st = ctypes.c_int
    c32p = ctypes.POINTER(QceC32)
    tp = ctypes.POINTER(QceTensor)
    i32p = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "qce_create": (st, [ctypes.POINTER(vp), ctypes.c_int]),
        "qce_destroy": (st, [vp]),
        "qce_set_stream": (st, [vp, vp]),
        "qce_set_mode": (st, [vp, ctypes.c_int]),
        "qce_get_mode": (st, [vp, ctypes.POINTER(ctypes.c_int)]),
        "qce_set_underflow_tolerance": (st, [vp, f64, f64]),
        "qce_set_size_policy": (st, [vp, i64, i64]),
        "qce_get_size_policy": (st, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "qce_set_gemm_size_policy": (st, [vp, i32]),
        "qce_set_gemm_tile": (st, [vp, i32]),
        "qce_set_workspace": (st, [vp, vp, ctypes.c_size_t]),
        "qce_cgemm_workspace_size": (ctypes.c_size_t, [i64, i64, i64]),
        "qce_cgemm_emulated": (st, [vp, ctypes.c_int, ctypes.c_int, i64, i64, i64, c32p, vp, i64,
                                    vp, i64, c32p, vp, i64]),
        "qce_cgemm_emulated_noalloc": (st, [vp, ctypes.c_int, ctypes.c_int, i64, i64, i64, c32p, vp, i64,
                                            vp, i64, c32p, vp, i64]),
        "qce_noalloc_scratch_bytes": (ctypes.c_size_t, []),
        "qce_get_last_decision": (st, [vp, ctypes.POINTER(QceDecision)]),
        "qce_cgemm_batched_workspace_size": (ctypes.c_size_t, [i64, i64, i64, i64]),
        "qce_cgemm_strided_batched": (st, [vp, ctypes.c_int, ctypes.c_int, i64, i64, i64, c32p, vp, i64, i64,
                                           vp, i64, i64, c32p, vp, i64, i64, i64]),
        "qce_cgemm_grouped": (st, [vp, i64, ctypes.POINTER(QceGemmDesc)]),
        "qce_get_batch_decision": (st, [vp, i64, ctypes.POINTER(QceDecision)]),
        "qce_contract": (st, [vp, tp, vp, i32p, tp, vp, i32p, tp, vp, i32p]),
        "qce_group_begin": (st, [vp]),
        "qce_group_end": (st, [vp]),
        "qce_group_reset": (st, [vp, ctypes.c_size_t]),
        "qce_permute": (st, [vp, tp, vp, i32p, vp]),
        "qce_accumulate_f64": (st, [vp, vp, vp]),
        "qce_accumulate_n_f64": (st, [vp, vp, i64, vp]),
        "qce_fidelity_f64": (st, [vp, vp, vp, i64, vp]),
        "qce_expstats": (st, [vp, vp, i64, i64, i64, ctypes.POINTER(QceDecision)]),
        "qce_split": (st, [vp, ctypes.c_int, i32, vp, i64, vp]),
        "qce_panel_bytes": (ctypes.c_size_t, [ctypes.c_int, i64, i64]),
        "qce_split_panels": (st, [vp, ctypes.c_int, i32, i32, i32, vp, i64, i64, i64, vp]),
        "qce_split_panels_bitmap": (st, [vp, ctypes.c_int, i32, vp, i32, i32, i32p, i32p, vp]),
        "qce_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "qce_last_error": (ctypes.c_char_p, [vp]),
        "qce_set_timing": (st, [vp, ctypes.c_int]),
        "qce_set_timing_tag": (st, [vp, i32]),
        "qce_reset_timing": (st, [vp]),
        "qce_get_timing": (st, [vp, i32, ctypes.POINTER(QceTiming)]),
    }
    for name in EXPORTS:
        fn = getattr(lib, name)
        fn.restype, fn.argtypes = sig[name]
    _lib = lib
    return lib
