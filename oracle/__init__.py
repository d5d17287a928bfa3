"""FP64 CPU oracle for NDGSBP decoding.

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the CPU
baseline leg of the benchmark may call it; the decoder library never does.
It shares no code with the HIP path. Pieces:

* ``ndgsbp_ref.c`` (built to ``libndgsbp_ref.so``): Steps 2-4 of Sec. II-C
  with eq. (1)-(3) in FP64, threaded over frames; also the vertical
  (VN-group) shuffled schedule that Sec. I cites as prior art.
* ``windows``: the contiguous CN windows with overlap (Python, below).
* ``literal``: a pure-Python version of the same schedule over a pluggable
  message algebra (real numbers or "which channel values reached here"
  sets), used on tiny graphs to pin the schedule to the paper's Fig. 1
  example.
* ``bitmap``: brute-force bitwise MAP over all codewords (tiny codes).

Parity status: every function here is pinned by tests under ``tests/``
(see ``test_oracle_*``); the clamp constant (30) is a definition shared with
the decoder, not something the paper fixes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ndgsbp_ref.c")
_LIB = os.path.join(_HERE, "libndgsbp_ref.so")
_lib = None

XMAX = 30.0


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, IEEE semantics kept: no -ffast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.ref_decode.restype = ctypes.c_int
        lib.ref_decode.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.c_int, i32p, i32p,
                                   ctypes.POINTER(ctypes.c_float), ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_uint8), i32p,
                                   ctypes.POINTER(ctypes.c_uint8), ctypes.c_int]
        lib.ref_decode_schedule.restype = ctypes.c_int
        lib.ref_decode_schedule.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.c_int, i32p, i32p,
                                            ctypes.c_int, ctypes.POINTER(ctypes.c_float), ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_uint8), i32p,
                                            ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_double),
                                            ctypes.c_int]
        lib.ref_decode_vertical.restype = ctypes.c_int
        lib.ref_decode_vertical.argtypes = lib.ref_decode.argtypes
        lib.ref_phi_f64.restype = ctypes.c_double
        lib.ref_phi_f64.argtypes = [ctypes.c_double]
        lib.ref_boxplus.restype = ctypes.c_double
        lib.ref_boxplus.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        _lib = lib
    return _lib


def windows(M: int, G: int, overlap: int, wrap: bool = True):
    """Contiguous CN windows (the grouping of Step 1 fixed to windows).

    Window g starts at floor(g*M/G) and ends just before the next window's
    start plus ``overlap`` CNs; with ``wrap`` the indices are taken mod M
    (so the last window overlaps the first), without it the last window
    stops at M."""
    out = []
    for g in range(G):
        start = (g * M) // G
        nxt = ((g + 1) * M) // G
        if wrap or g < G - 1:
            length = nxt - start + overlap
        else:
            length = M - start
        if length > M:
            raise ValueError("window longer than M")
        idx = [(start + i) % M for i in range(length)] if wrap else \
              [start + i for i in range(length) if start + i < M]
        out.append(np.array(idx, dtype=np.int32))
    return out


def _groups_csr(groups):
    gptr = np.zeros(len(groups) + 1, dtype=np.int32)
    gptr[1:] = np.cumsum([len(g) for g in groups])
    gcn = np.concatenate([np.asarray(g, dtype=np.int32) for g in groups]) if groups else \
        np.zeros(0, np.int32)
    return gptr, np.ascontiguousarray(gcn, dtype=np.int32)


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def decode(code, groups, llr, max_iter: int, early_stop: bool, nthreads: int = 0,
           groups_per_iteration: int = 0):
    """Run the FP64 oracle on float32 LLRs (F x n).

    ``code`` has m, n, row_ptr, col_idx; ``groups`` is a list of CN-id arrays
    processed in order. With ``groups_per_iteration`` = Gp > 0 the groups
    form blocks of Gp and iteration l uses block (l-1) mod (len(groups)/Gp)
    (a new grouping every iteration, Step 4 back to Step 1). Returns
    dict(post=float64 (F,n), hard=uint8 (F,n), iters=int32 (F,),
    syn_ok=uint8 (F,), margin=float64 (F,), threads=int); ``margin`` is
    the stop margin: the smallest change of total LLRs that could move the
    iteration at which the syndrome test of Step 4 stops the frame (minimum
    over iterations of: with a zero syndrome, the smallest |P| of a VN in
    some check; otherwise the largest over failing checks of the smallest
    |P| in the check)."""
    lib = _load()
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    if llr.ndim == 1:
        llr = llr[None, :]
    F, n = llr.shape
    assert n == code.n
    row_ptr = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    gptr, gcn = _groups_csr(groups)
    post = np.zeros((F, n), dtype=np.float64)
    hard = np.zeros((F, n), dtype=np.uint8)
    iters = np.zeros(F, dtype=np.int32)
    syn = np.zeros(F, dtype=np.uint8)
    margin = np.zeros(F, dtype=np.float64)
    i32 = ctypes.c_int32
    rc = lib.ref_decode_schedule(code.m, n, _p(row_ptr, i32), _p(col, i32), len(groups), _p(gptr, i32),
                        _p(gcn, i32), int(groups_per_iteration), _p(llr, ctypes.c_float), F, int(max_iter),
                        int(bool(early_stop)),
                        _p(post, ctypes.c_double), _p(hard, ctypes.c_uint8), _p(iters, i32),
                        _p(syn, ctypes.c_uint8), _p(margin, ctypes.c_double), int(nthreads))
    if rc < 0:
        raise ValueError(f"ref_decode rejected its input ({rc})")
    return dict(post=post, hard=hard, iters=iters, syn_ok=syn, margin=margin, threads=rc)


def decode_vertical(code, vn_groups, llr, max_iter: int, early_stop: bool, nthreads: int = 0):
    """Vertical group-shuffled decoding (the prior-art schedule Sec. I
    contrasts with: VN groups processed in order; for each, the CN->VN
    messages into its VNs from the VN->CN messages as they stood before the
    group, eq. (1), then those VNs' VN->CN messages, eq. (2)). Same inputs
    and outputs as ``decode`` with VN-id groups."""
    lib = _load()
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    if llr.ndim == 1:
        llr = llr[None, :]
    F, n = llr.shape
    assert n == code.n
    row_ptr = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    gptr, gvn = _groups_csr(vn_groups)
    post = np.zeros((F, n), dtype=np.float64)
    hard = np.zeros((F, n), dtype=np.uint8)
    iters = np.zeros(F, dtype=np.int32)
    syn = np.zeros(F, dtype=np.uint8)
    i32 = ctypes.c_int32
    rc = lib.ref_decode_vertical(code.m, n, _p(row_ptr, i32), _p(col, i32), len(vn_groups), _p(gptr, i32),
                                 _p(gvn, i32), _p(llr, ctypes.c_float), F, int(max_iter), int(bool(early_stop)),
                                 _p(post, ctypes.c_double), _p(hard, ctypes.c_uint8), _p(iters, i32),
                                 _p(syn, ctypes.c_uint8), int(nthreads))
    if rc < 0:
        raise ValueError(f"ref_decode_vertical rejected its input ({rc})")
    return dict(post=post, hard=hard, iters=iters, syn_ok=syn, threads=rc)


def decode_vertical_with_sensitivity(code, vn_groups, llr, max_iter: int, early_stop: bool, nthreads: int = 0):
    """decode_vertical plus the one-ulp sensitivity of decode_with_sensitivity."""
    ref = decode_vertical(code, vn_groups, llr, max_iter, early_stop, nthreads)
    ctl = decode_vertical(code, vn_groups, perturb_one_ulp(llr), max_iter, early_stop, nthreads)
    sens = np.abs(ctl["post"] - ref["post"]).max(axis=1)
    flip = np.any(ctl["hard"] != ref["hard"], axis=1) | (ctl["iters"] != ref["iters"])
    sens[flip] = np.inf
    ref["sens"] = sens
    return ref


def perturb_one_ulp(llr, seed: int = 12345):
    """The same float32 LLRs, each moved by one ulp up or down (seeded)."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    d = np.random.default_rng(seed).choice(np.array([-np.inf, np.inf], np.float32), size=llr.shape)
    return np.nextafter(llr, d).astype(np.float32)


def decode_with_sensitivity(code, groups, llr, max_iter: int, early_stop: bool, nthreads: int = 0,
                            groups_per_iteration: int = 0):
    """Oracle result plus each frame's conditioning: ``sens[f]`` is the largest
    posterior change when every input LLR moves by one float32 ulp (inf when
    that already changes a hard decision). It measures how strongly the FP64
    decode amplifies rounding-sized input changes on that frame."""
    ref = decode(code, groups, llr, max_iter, early_stop, nthreads, groups_per_iteration)
    ctl = decode(code, groups, perturb_one_ulp(llr), max_iter, early_stop, nthreads, groups_per_iteration)
    sens = np.abs(ctl["post"] - ref["post"]).max(axis=1)
    flip = np.any(ctl["hard"] != ref["hard"], axis=1) | (ctl["iters"] != ref["iters"])
    sens[flip] = np.inf
    ref["sens"] = sens
    llr = np.ascontiguousarray(llr, dtype=np.float32).reshape(-1, code.n)

    def rerun(frames, iters):
        """Posteriors of the given frames after exactly iters[i] iterations
        (no early stop): the oracle's result at another stop iteration."""
        frames = np.asarray(frames, dtype=np.int64)
        iters = np.asarray(iters, dtype=np.int64)
        out = np.zeros((len(frames), code.n))
        for it in np.unique(iters):
            sel = np.nonzero(iters == it)[0]
            out[sel] = decode(code, groups, llr[frames[sel]], int(it), False, nthreads,
                              groups_per_iteration)["post"]
        return out

    ref["rerun"] = rerun
    return ref


def phi(x: float) -> float:
    return _load().ref_phi_f64(float(x))


def boxplus(xs) -> float:
    a = np.ascontiguousarray(xs, dtype=np.float64)
    return _load().ref_boxplus(_p(a, ctypes.c_double), len(a))
