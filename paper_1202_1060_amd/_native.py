"""ctypes declarations of the C ABI in include/ndgsbp.h (libndgsbp.so).

Loading fails loudly when the library has not been built; there is no
fallback decoder in this package.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libndgsbp.so")

LDPC_OK = 0
LDPC_EINVAL = -1
LDPC_ENOMEM = -2
LDPC_EHIP = -3
LDPC_EUNSUPPORTED = -4

LDPC_GROUPS_WINDOWS = 0
LDPC_GROUPS_EXPLICIT = 1
LDPC_GROUPS_VN = 2

LDPC_FLAG_EARLY_STOP = 0x1
LDPC_FLAG_MSG_FP16 = 0x2
LDPC_FLAG_MSG_BF16 = 0x4
LDPC_FLAG_OUT_PACKED = 0x8
LDPC_FLAG_TIER_HBM = 0x10

EXPORTS = ("ldpc_code_create", "ldpc_code_destroy", "ldpc_code_query", "ldpc_code_tune",
           "ldpc_decode", "ldpc_decode_noalloc", "ldpc_batch_create", "ldpc_batch_launch", "ldpc_batch_query",
           "ldpc_batch_destroy", "ldpc_decode_batched", "ldpc_last_error")

_i32p = ctypes.POINTER(ctypes.c_int32)


class ldpc_h_csr(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", _i32p), ("col_idx", _i32p)]


class ldpc_grouping(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("num_groups", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("wrap", ctypes.c_int32),
                ("group_ptr", _i32p), ("group_cn", _i32p), ("groups_per_iteration", ctypes.c_int32)]


class ldpc_code_info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("num_groups", ctypes.c_int32), ("cn_visits", ctypes.c_int64),
                ("edge_updates", ctypes.c_int64), ("max_cn_degree", ctypes.c_int32),
                ("max_vn_degree", ctypes.c_int32), ("device", ctypes.c_int32),
                ("lds_bytes_fp32", ctypes.c_int64), ("lds_bytes_16", ctypes.c_int64),
                ("lds_limit", ctypes.c_int64), ("lanes_fp32", ctypes.c_int32), ("lanes_fp16", ctypes.c_int32),
                ("lanes_bf16", ctypes.c_int32), ("groups_per_iteration", ctypes.c_int32)]


class ldpc_problem(ctypes.Structure):
    _fields_ = [("code", ctypes.c_void_p), ("llr", ctypes.c_void_p), ("num_frames", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("hard", ctypes.c_void_p), ("post", ctypes.c_void_p),
                ("iters", ctypes.c_void_p), ("syn_ok", ctypes.c_void_p)]


class ldpc_batch_options(ctypes.Structure):
    _fields_ = [("lanes_per_cn", ctypes.c_int32), ("split_by_size", ctypes.c_int32),
                ("max_threads", ctypes.c_int32), ("streams", ctypes.c_int32)]


class ldpc_batch_info(ctypes.Structure):
    _fields_ = [("num_launches", ctypes.c_int32), ("num_problems", ctypes.c_int32),
                ("num_streams", ctypes.c_int32), ("total_frames", ctypes.c_int64)]


class LdpcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libndgsbp.so (torch must already be imported, so that the
    library binds to the HIP runtime torch loaded)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python -m paper_1202_1060_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.ldpc_code_create.restype = ctypes.c_int
    lib.ldpc_code_create.argtypes = [ctypes.POINTER(ldpc_h_csr), ctypes.POINTER(ldpc_grouping),
                                     ctypes.c_int32, ctypes.POINTER(vp)]
    lib.ldpc_code_destroy.restype = ctypes.c_int
    lib.ldpc_code_destroy.argtypes = [vp]
    lib.ldpc_code_query.restype = ctypes.c_int
    lib.ldpc_code_query.argtypes = [vp, ctypes.POINTER(ldpc_code_info)]
    lib.ldpc_code_tune.restype = ctypes.c_int
    lib.ldpc_code_tune.argtypes = [vp, ctypes.c_uint32, ctypes.c_int32]
    lib.ldpc_decode.restype = ctypes.c_int
    lib.ldpc_decode.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                vp, vp, vp, vp, vp]
    lib.ldpc_decode_noalloc.restype = ctypes.c_int
    lib.ldpc_decode_noalloc.argtypes = lib.ldpc_decode.argtypes
    lib.ldpc_batch_create.restype = ctypes.c_int
    lib.ldpc_batch_create.argtypes = [ctypes.POINTER(ldpc_problem), ctypes.c_int32, ctypes.c_uint32,
                                      ctypes.POINTER(ldpc_batch_options), ctypes.POINTER(vp)]
    lib.ldpc_batch_launch.restype = ctypes.c_int
    lib.ldpc_batch_launch.argtypes = [vp, vp]
    lib.ldpc_batch_query.restype = ctypes.c_int
    lib.ldpc_batch_query.argtypes = [vp, ctypes.POINTER(ldpc_batch_info)]
    lib.ldpc_batch_destroy.restype = ctypes.c_int
    lib.ldpc_batch_destroy.argtypes = [vp]
    lib.ldpc_decode_batched.restype = ctypes.c_int
    lib.ldpc_decode_batched.argtypes = [ctypes.POINTER(ldpc_problem), ctypes.c_int32, ctypes.c_uint32, vp]
    lib.ldpc_last_error.restype = ctypes.c_char_p
    lib.ldpc_last_error.argtypes = []
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != LDPC_OK:
        msg = load().ldpc_last_error().decode(errors="replace")
        raise LdpcError(rc, msg or "ldpc call failed")
