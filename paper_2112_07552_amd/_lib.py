"""ctypes binding of libtcudb.so (include/tcudb.h), argument marshalling only.

Every step of the operator runs in the library's HIP kernels; this module
only turns torch tensors into device pointers and the caller's current HIP
stream.  There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtcudb.so")

TCU_OK = 0
TCU_ERR_ARG = -1
TCU_ERR_KEY_RANGE = -2
TCU_ERR_WORKSPACE = -3
TCU_ERR_INFEASIBLE = -4
TCU_ERR_NONFINITE = -5
TCU_ERR_HIP = -6
TCU_ERR_COUNT_RANGE = -7

TCU_F64 = 0
TCU_F32 = 1

TCU_PREC_FP64 = 0
TCU_PREC_SPLIT_BF16 = 1
TCU_PREC_SPLIT_I8 = 2
TCU_PREC_CRT_I8 = 3
TCU_MAX_SLICES = 8
TCU_MAX_MODULI = 15

TCU_FLAG_KEY_RANGE = 1
TCU_FLAG_NONFINITE = 2
TCU_FLAG_FALLBACK = 4
TCU_FLAG_COUNT_RANGE = 8
NEED_UNCERTIFIED = 255

TCU_WS_BACKWARD = 1
TCU_WS_COUNT = 2

TCU_REL_UNIQUE_CELLS = 1
TCU_NOALLOC_MAX_BYTES = (64 << 20) + (64 << 10)
TCU_BWD_SAVED_ENCODINGS = 1

EXPORTS = (
    "tcu_workspace_bytes", "tcu_mixed_plan", "tcu_split", "tcu_encode",
    "tcu_encode_workspace_bytes", "tcu_gemm_f64",
    "tcu_gemm_f64_workspace_bytes", "tcu_gemm_f64_ws",
    "tcu_join_agg_fwd", "tcu_join_agg_fwd_noalloc", "tcu_join_agg_bwd", "tcu_dict_workspace_bytes", "tcu_dict_encode",
    "tcu_join_agg_row_workspace_bytes", "tcu_join_agg_row",
    "tcu_join_agg_bsr_workspace_bytes", "tcu_join_agg_bsr", "tcu_block_sparse_preferred",
    "tcu_nonzero_workspace_bytes",
    "tcu_nonzero", "tcu_gemm_f64_host", "tcu_mfma_peak_out_bytes", "tcu_mfma_peak_ops",
    "tcu_mfma_peak", "tcu_trace_launches", "tcu_sync_status",
    "tcu_status_str", "tcu_version",
)


class tcu_relation(C.Structure):
    _fields_ = [("n", C.c_int64), ("group", C.c_void_p), ("key", C.c_void_p),
                ("val", C.c_void_p), ("dtype", C.c_int), ("flags", C.c_uint32)]


class tcu_status_info(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("slices", C.c_uint32),
                ("skipped_a", C.c_uint64), ("skipped_b", C.c_uint64),
                ("bits", C.c_uint32), ("need", C.c_uint32), ("exceptions", C.c_uint32)]


TCU_KERNEL_GEMM_F64 = 1
TCU_KERNEL_GEMM_CRT = 2
TCU_KERNEL_CERTIFY = 3
TCU_KERNEL_GEMM_SPLIT = 4
TCU_KERNEL_ENCODE = 5
TCU_KERNEL_GATHER = 6
TCU_KERNEL_COUNT = 7


class tcu_launch_record(C.Structure):
    _fields_ = [("begin", C.c_void_p), ("end", C.c_void_p), ("kernel", C.c_int32),
                ("m", C.c_int32), ("n", C.c_int32), ("k", C.c_int32), ("planes", C.c_int32),
                ("ops", C.c_double)]


class TcuError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})" if what else status_str(status))


_lib = None


def load():
    """Load libtcudb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    rel_p = C.POINTER(tcu_relation)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.tcu_workspace_bytes.argtypes = [rel_p, rel_p, i32, i32, i32, C.c_int, C.c_int]
    L.tcu_workspace_bytes.restype = C.c_size_t
    L.tcu_mixed_plan.argtypes = [C.c_int, i32, f64, C.c_uint32, f64, C.POINTER(C.c_int32)]
    L.tcu_mixed_plan.restype = C.c_int
    L.tcu_split.argtypes = [vp, i32, i32, i64, C.c_int, C.c_int, i32, vp, i32, i32, vp, vp,
                            C.c_size_t, vp]
    L.tcu_split.restype = C.c_int
    L.tcu_encode.argtypes = [rel_p, C.c_int, i32, i32, vp, vp, C.c_size_t, vp]
    L.tcu_encode.restype = C.c_int
    L.tcu_encode_workspace_bytes.argtypes = [rel_p, i32, i32]
    L.tcu_encode_workspace_bytes.restype = C.c_size_t
    L.tcu_gemm_f64.argtypes = [C.c_int, C.c_int, i32, i32, i32, vp, i64, vp, i64, vp, i64, vp]
    L.tcu_gemm_f64.restype = C.c_int
    L.tcu_gemm_f64_workspace_bytes.argtypes = [i32, i32, i32]
    L.tcu_gemm_f64_workspace_bytes.restype = C.c_size_t
    L.tcu_gemm_f64_ws.argtypes = [C.c_int, C.c_int, i32, i32, i32, vp, i64, vp, i64, vp, i64, vp,
                                  C.c_size_t, vp]
    L.tcu_gemm_f64_ws.restype = C.c_int
    L.tcu_join_agg_fwd.argtypes = [rel_p, rel_p, i32, i32, i32, C.c_int, f64, vp, vp, vp,
                                   C.c_size_t, vp]
    L.tcu_join_agg_fwd.restype = C.c_int
    L.tcu_join_agg_fwd_noalloc.argtypes = [rel_p, rel_p, i32, i32, i32, C.c_int, f64, vp, vp,
                                           vp, vp]
    L.tcu_join_agg_fwd_noalloc.restype = C.c_int
    L.tcu_join_agg_bwd.argtypes = [rel_p, rel_p, i32, i32, i32, C.c_int, f64, vp, vp, vp,
                                   C.c_int, vp, C.c_size_t, vp]
    L.tcu_join_agg_bwd.restype = C.c_int
    L.tcu_dict_workspace_bytes.argtypes = [i64]
    L.tcu_dict_workspace_bytes.restype = C.c_size_t
    L.tcu_dict_encode.argtypes = [vp, i64, vp, i64, vp, vp, vp, C.POINTER(C.c_int64), vp,
                                  C.c_size_t, vp]
    L.tcu_dict_encode.restype = C.c_int
    L.tcu_join_agg_row_workspace_bytes.argtypes = [i32, i32]
    L.tcu_join_agg_row_workspace_bytes.restype = C.c_size_t
    L.tcu_join_agg_row.argtypes = [rel_p, rel_p, i32, i32, vp, vp, vp, C.c_size_t, vp]
    L.tcu_join_agg_row.restype = C.c_int
    L.tcu_join_agg_bsr_workspace_bytes.argtypes = [rel_p, rel_p, i32, i32, i32]
    L.tcu_join_agg_bsr_workspace_bytes.restype = C.c_size_t
    L.tcu_join_agg_bsr.argtypes = [rel_p, rel_p, i32, i32, i32, vp, vp, C.c_size_t, vp]
    L.tcu_join_agg_bsr.restype = C.c_int
    L.tcu_block_sparse_preferred.argtypes = [rel_p, rel_p, i32, i32, i32]
    L.tcu_block_sparse_preferred.restype = C.c_int
    L.tcu_nonzero_workspace_bytes.argtypes = [i64, i64]
    L.tcu_nonzero_workspace_bytes.restype = C.c_size_t
    L.tcu_nonzero.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, i64, C.POINTER(C.c_int64), vp,
                              C.c_size_t, vp]
    L.tcu_nonzero.restype = C.c_int
    L.tcu_gemm_f64_host.argtypes = [i32, i32, i32, vp, i64, vp, i64, vp, i64, vp, C.c_size_t,
                                    i64, vp]
    L.tcu_gemm_f64_host.restype = C.c_int
    L.tcu_mfma_peak_out_bytes.argtypes = []
    L.tcu_mfma_peak_out_bytes.restype = C.c_size_t
    L.tcu_mfma_peak_ops.argtypes = [C.c_int, i32]
    L.tcu_mfma_peak_ops.restype = f64
    L.tcu_mfma_peak.argtypes = [C.c_int, i32, vp, vp]
    L.tcu_mfma_peak.restype = C.c_int
    L.tcu_trace_launches.argtypes = [C.POINTER(tcu_launch_record), i32, C.POINTER(C.c_int32)]
    L.tcu_trace_launches.restype = C.c_int
    L.tcu_sync_status.argtypes = [vp, vp, C.POINTER(tcu_status_info)]
    L.tcu_sync_status.restype = C.c_int
    L.tcu_status_str.argtypes = [C.c_int]
    L.tcu_status_str.restype = C.c_char_p
    L.tcu_version.argtypes = []
    L.tcu_version.restype = C.c_char_p
    _lib = L
    return L


def status_str(status: int) -> str:
    try:
        return load().tcu_status_str(status).decode()
    except RuntimeError:
        return f"status {status}"


def check(status: int, what: str) -> None:
    if status != TCU_OK:
        raise TcuError(status, what)
