"""MI355X (gfx950) NDGSBP LDPC decoder: thin Python binding of libndgsbp.so.

The functions keep the C names (``ldpc_code_create``, ``ldpc_decode`` ...)
and only marshal arguments; every step of the decode runs in the HIP
kernels. PyTorch supplies device memory and streams. Importing this package
imports torch first so that the library binds to the HIP runtime torch has
loaded.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch  # noqa: F401  (must precede loading the library)

from . import _native
from ._native import (LdpcError, LDPC_OK, LDPC_EINVAL, LDPC_ENOMEM, LDPC_EHIP,
                      LDPC_EUNSUPPORTED, LDPC_GROUPS_WINDOWS, LDPC_GROUPS_EXPLICIT,
                      LDPC_FLAG_EARLY_STOP, LDPC_FLAG_MSG_FP16, LDPC_FLAG_MSG_BF16,
                      LDPC_FLAG_OUT_PACKED)

__all__ = [
    "Code", "ldpc_code_create", "ldpc_code_destroy", "ldpc_code_query", "ldpc_code_tune", "ldpc_decode",
    "ldpc_decode_noalloc",
    "ldpc_batch_create", "ldpc_batch_launch", "ldpc_batch_query", "ldpc_batch_destroy",
    "ldpc_decode_batched", "Problem", "Batch", "BatchOptions", "decode_batched", "new_outputs",
    "ldpc_last_error", "decode", "LdpcError", "msg_flag",
    "LDPC_FLAG_EARLY_STOP", "LDPC_FLAG_MSG_FP16", "LDPC_FLAG_MSG_BF16", "LDPC_FLAG_OUT_PACKED",
]



def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def ldpc_last_error() -> str:
    return _native.load().ldpc_last_error().decode(errors="replace")


def ldpc_code_create(m, n, row_ptr, col_idx, *, windows=None, groups=None, vn_groups=None, device=0,
                     groups_per_iteration=0):
    """Create a device code handle (see include/ndgsbp.h).

    ``windows=(G, overlap, wrap)`` or ``groups=[CN-id arrays]`` (in order;
    with ``groups_per_iteration`` = Gp, iteration l uses the l-th block of
    Gp groups, cyclically), or ``vn_groups=[VN-id arrays]`` for the vertical
    group-shuffled schedule. Returns the opaque handle (int)."""
    rp, ci = _i32(row_ptr), _i32(col_idx)
    h = _native.ldpc_h_csr(int(m), int(n), int(len(ci)), _ptr(rp), _ptr(ci))
    if sum(x is not None for x in (windows, groups, vn_groups)) != 1:
        raise ValueError("give exactly one of windows=, groups= or vn_groups=")
    keep = []
    if windows is not None:
        G, o, wrap = windows
        g = _native.ldpc_grouping(LDPC_GROUPS_WINDOWS, int(G), int(o), int(bool(wrap)), None, None, 0)
    else:
        lists = groups if groups is not None else vn_groups
        gptr = _i32(np.concatenate([[0], np.cumsum([len(x) for x in lists])]))
        gcn = _i32(np.concatenate([np.asarray(x) for x in lists]) if len(lists) else [])
        keep += [gptr, gcn]
        kind = LDPC_GROUPS_EXPLICIT if groups is not None else _native.LDPC_GROUPS_VN
        g = _native.ldpc_grouping(kind, len(lists), 0, 0, _ptr(gptr), _ptr(gcn), int(groups_per_iteration))
    out = ctypes.c_void_p()
    _native.check(_native.load().ldpc_code_create(ctypes.byref(h), ctypes.byref(g), int(device), ctypes.byref(out)))
    return out.value


def ldpc_code_destroy(handle) -> None:
    _native.check(_native.load().ldpc_code_destroy(ctypes.c_void_p(handle)))


def ldpc_code_query(handle) -> dict:
    info = _native.ldpc_code_info()
    _native.check(_native.load().ldpc_code_query(ctypes.c_void_p(handle), ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in info._fields_}


def ldpc_code_tune(handle, msg_flags: int, lanes_per_cn: int) -> None:
    _native.check(_native.load().ldpc_code_tune(ctypes.c_void_p(handle), int(msg_flags), int(lanes_per_cn)))


def ldpc_decode(handle, llr_ptr, num_frames, max_iter, flags, hard_ptr, post_ptr, iters_ptr,
                syn_ok_ptr, stream) -> None:
    """Raw entry point: device pointers as ints (0 for NULL), stream handle as int."""
    _native.check(_native.load().ldpc_decode(ctypes.c_void_p(handle), ctypes.c_void_p(llr_ptr),
                                   int(num_frames), int(max_iter), int(flags),
                                   ctypes.c_void_p(hard_ptr), ctypes.c_void_p(post_ptr or None),
                                   ctypes.c_void_p(iters_ptr), ctypes.c_void_p(syn_ok_ptr or None),
                                   ctypes.c_void_p(stream or None)))


def ldpc_decode_noalloc(handle, llr_ptr, num_frames, max_iter, flags, hard_ptr, post_ptr, iters_ptr,
                        syn_ok_ptr, stream) -> None:
    """ldpc_decode without allocation (fixed per-GPU scratch); same arguments."""
    _native.check(_native.load().ldpc_decode_noalloc(ctypes.c_void_p(handle), ctypes.c_void_p(llr_ptr),
                                                     int(num_frames), int(max_iter), int(flags),
                                                     ctypes.c_void_p(hard_ptr), ctypes.c_void_p(post_ptr or None),
                                                     ctypes.c_void_p(iters_ptr),
                                                     ctypes.c_void_p(syn_ok_ptr or None),
                                                     ctypes.c_void_p(stream or None)))


def msg_flag(msg: str) -> int:
    return {"fp32": 0, "fp16": LDPC_FLAG_MSG_FP16, "bf16": LDPC_FLAG_MSG_BF16}[msg]


class Code:
    """Owns a device code handle. ``code`` is any object with m, n, row_ptr,
    col_idx (e.g. ldpcgen.Code)."""

    def __init__(self, code, *, windows=None, groups=None, vn_groups=None, device=0, groups_per_iteration=0):
        self.m, self.n = int(code.m), int(code.n)
        self.handle = ldpc_code_create(code.m, code.n, code.row_ptr, code.col_idx,
                                       windows=windows, groups=groups, vn_groups=vn_groups, device=device,
                                       groups_per_iteration=groups_per_iteration)
        self.info = ldpc_code_query(self.handle)
        self.device = device

    def tune(self, msg: str, lanes_per_cn: int) -> None:
        """Pick the CN-phase mapping (1, 2 or 4 lanes per CN visit, 0 = default)
        used by decodes with message format ``msg``."""
        ldpc_code_tune(self.handle, msg_flag(msg), lanes_per_cn)
        self.info = ldpc_code_query(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            ldpc_code_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode(code: Code, llr: torch.Tensor, max_iter: int, *, early_stop: bool = True,
           msg: str = "fp32", want_post: bool = True, want_syn: bool = True, out=None,
           stream=None, packed: bool = False):
    """Decode a (F, n) float32 device tensor; returns dict of device tensors
    hard (uint8, (F, n), or (F, ceil(n/8)) bit-packed LSB first with
    ``packed``), post (float32, optional), iters (int32), syn_ok (uint8)."""
    if llr.dtype != torch.float32 or llr.dim() != 2 or llr.shape[1] != code.n:
        raise ValueError("llr must be a (F, n) float32 tensor")
    if not llr.is_cuda or not llr.is_contiguous():
        raise ValueError("llr must be a contiguous device tensor")
    F = llr.shape[0]
    dev = llr.device
    if out is None:
        out = new_outputs(F, code.n, dev, want_post, want_syn, packed)
    _check_outputs(out, F, code.n, packed)
    flags = msg_flag(msg) | (LDPC_FLAG_EARLY_STOP if early_stop else 0) | (LDPC_FLAG_OUT_PACKED if packed else 0)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    ldpc_decode(code.handle, llr.data_ptr(), F, max_iter, flags, out["hard"].data_ptr(),
                out["post"].data_ptr() if out.get("post") is not None else 0,
                out["iters"].data_ptr(),
                out["syn_ok"].data_ptr() if out.get("syn_ok") is not None else 0,
                s.cuda_stream)
    return out


# ---- batched decoding ------------------------------------------------------

class BatchOptions:
    """Launch choices of a batch (ldpc_batch_options). Defaults: each code's
    CN-lane mapping, one launch per LDS size class, workgroups sized for the
    largest group, four streams."""

    __slots__ = ("lanes_per_cn", "split_by_size", "max_threads", "streams")

    def __init__(self, lanes_per_cn=0, split_by_size=1, max_threads=0, streams=4):
        self.lanes_per_cn = int(lanes_per_cn)
        self.split_by_size = int(split_by_size)
        self.max_threads = int(max_threads)
        self.streams = int(streams)

    def as_tuple(self):
        return (self.lanes_per_cn, self.split_by_size, self.max_threads, self.streams)

    @classmethod
    def from_tuple(cls, t):
        return cls(*t)

    def __repr__(self):
        return "BatchOptions(lanes_per_cn=%d, split_by_size=%d, max_threads=%d, streams=%d)" % self.as_tuple()

    def _c(self):
        return _native.ldpc_batch_options(*self.as_tuple())


def hard_width(n: int, packed: bool) -> int:
    return (n + 7) // 8 if packed else n


def _check_outputs(out, F, n, packed):
    for k in ("hard", "post", "iters", "syn_ok"):
        t = out.get(k)
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("%s must be a contiguous device tensor" % k)
    if tuple(out["hard"].shape) != (F, hard_width(n, packed)) or out["hard"].dtype != torch.uint8:
        raise ValueError("hard must be a (F, %d) uint8 tensor" % hard_width(n, packed))
    if tuple(out["iters"].shape) != (F,) or out["iters"].dtype != torch.int32:
        raise ValueError("iters must be a (F,) int32 tensor")
    if out.get("post") is not None and (tuple(out["post"].shape) != (F, n) or out["post"].dtype != torch.float32):
        raise ValueError("post must be a (F, n) float32 tensor")
    if out.get("syn_ok") is not None and (tuple(out["syn_ok"].shape) != (F,) or out["syn_ok"].dtype != torch.uint8):
        raise ValueError("syn_ok must be a (F,) uint8 tensor")


def new_outputs(F: int, n: int, device, want_post=True, want_syn=True, packed=False) -> dict:
    return dict(hard=torch.empty((F, hard_width(n, packed)), dtype=torch.uint8, device=device),
                post=torch.empty((F, n), dtype=torch.float32, device=device) if want_post else None,
                iters=torch.empty((F,), dtype=torch.int32, device=device),
                syn_ok=torch.empty((F,), dtype=torch.uint8, device=device) if want_syn else None)


class Problem:
    """One problem of a batch: a Code, a (F, n) float32 device tensor of
    channel LLRs, an iteration cap and the output tensors (allocated here
    unless given)."""

    def __init__(self, code: Code, llr: torch.Tensor, max_iter: int, *, out=None, want_post=True,
                 want_syn=True, packed=False):
        if llr.dtype != torch.float32 or llr.dim() != 2 or llr.shape[1] != code.n:
            raise ValueError("llr must be a (F, n) float32 tensor")
        if not llr.is_cuda or not llr.is_contiguous():
            raise ValueError("llr must be a contiguous device tensor")
        self.code, self.llr, self.max_iter, self.packed = code, llr, int(max_iter), bool(packed)
        self.out = out if out is not None else new_outputs(llr.shape[0], code.n, llr.device, want_post, want_syn,
                                                           packed)
        _check_outputs(self.out, llr.shape[0], code.n, packed)

    def _c(self):
        o = self.out
        return _native.ldpc_problem(self.code.handle, self.llr.data_ptr(), int(self.llr.shape[0]),
                                    self.max_iter, o["hard"].data_ptr(),
                                    o["post"].data_ptr() if o.get("post") is not None else None,
                                    o["iters"].data_ptr(),
                                    o["syn_ok"].data_ptr() if o.get("syn_ok") is not None else None)


def _batch_flags(problems, msg, early_stop):
    packed = {p.packed for p in problems}
    if len(packed) > 1:
        raise ValueError("all problems of a batch must use the same hard-decision layout")
    return (msg_flag(msg) | (LDPC_FLAG_EARLY_STOP if early_stop else 0)
            | (LDPC_FLAG_OUT_PACKED if packed == {True} else 0))


def _problem_array(problems):
    arr = (_native.ldpc_problem * max(1, len(problems)))()
    for i, p in enumerate(problems):
        arr[i] = p._c()
    return arr


def ldpc_batch_create(problems, flags: int, options: BatchOptions | None = None):
    arr = _problem_array(problems)
    out = ctypes.c_void_p()
    opt = options._c() if options is not None else None
    _native.check(_native.load().ldpc_batch_create(arr, len(problems), int(flags),
                                                   ctypes.byref(opt) if opt is not None else None,
                                                   ctypes.byref(out)))
    return out.value


def ldpc_batch_launch(handle, stream) -> None:
    _native.check(_native.load().ldpc_batch_launch(ctypes.c_void_p(handle), ctypes.c_void_p(stream or None)))


def ldpc_batch_query(handle) -> dict:
    info = _native.ldpc_batch_info()
    _native.check(_native.load().ldpc_batch_query(ctypes.c_void_p(handle), ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in info._fields_}


def ldpc_batch_destroy(handle) -> None:
    _native.check(_native.load().ldpc_batch_destroy(ctypes.c_void_p(handle)))


def ldpc_decode_batched(problems, flags: int, stream) -> None:
    arr = _problem_array(problems)
    _native.check(_native.load().ldpc_decode_batched(arr, len(problems), int(flags),
                                                     ctypes.c_void_p(stream or None)))


class Batch:
    """A batch plan (ldpc_batch_*): created once, launched any number of
    times (also inside a CUDA/HIP graph capture), each launch decoding every
    problem's current LLR tensor into its output tensors."""

    def __init__(self, problems, *, msg="fp16", early_stop=True, options: BatchOptions | None = None):
        self.problems = list(problems)
        self.flags = _batch_flags(self.problems, msg, early_stop)
        self.handle = ldpc_batch_create(self.problems, self.flags, options)
        self.info = ldpc_batch_query(self.handle)

    def launch(self, stream=None):
        dev = self.problems[0].llr.device if self.problems else torch.device("cuda", 0)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        ldpc_batch_launch(self.handle, s.cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            ldpc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode_batched(problems, *, msg="fp16", early_stop=True, stream=None):
    """One-shot batched decode (ldpc_decode_batched), asynchronous on
    ``stream``; returns the problems' output dicts."""
    flags = _batch_flags(problems, msg, early_stop)
    dev = problems[0].llr.device if problems else torch.device("cuda", 0)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    ldpc_decode_batched(problems, flags, s.cuda_stream)
    return [p.out for p in problems]
