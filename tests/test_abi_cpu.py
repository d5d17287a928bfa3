"""C ABI checks that need no GPU: the library loads, exports every symbol
the header declares, and rejects malformed input before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ndgsbp.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*|void)\s+(ldpc_\w+)\s*\(", src, re.M)))


def test_header_declares_the_abi():
    assert _declared() == sorted(["ldpc_code_create", "ldpc_code_destroy", "ldpc_code_query",
                                  "ldpc_code_tune", "ldpc_decode", "ldpc_decode_noalloc", "ldpc_batch_create",
                                  "ldpc_batch_launch", "ldpc_batch_query", "ldpc_batch_destroy",
                                  "ldpc_decode_batched", "ldpc_last_error"])


def test_library_exports_every_declared_symbol():
    from paper_1202_1060_amd import _native
    assert os.path.exists(_native.LIB_PATH), "build the library first"
    out = subprocess.run(["nm", "-D", "--defined-only", _native.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (ldpc_\w+)", out))
    for sym in _declared():
        assert sym in exported, sym
    assert set(_native.EXPORTS) == set(_declared())


def test_header_compiles_as_c():
    src = '#include "ndgsbp.h"\nint main(void){ldpc_code_t c = 0; (void)c; return LDPC_OK;}\n'
    res = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                          "-x", "c", "-", "-o", "/dev/null"], input=src, text=True, capture_output=True)
    assert res.returncode == 0, res.stderr


@pytest.fixture(scope="module")
def nd():
    import paper_1202_1060_amd as mod
    return mod


def _create(nd, m, n, row_ptr, col, windows=(1, 0, 0), groups=None):
    if groups is not None:
        return nd.ldpc_code_create(m, n, row_ptr, col, groups=groups)
    return nd.ldpc_code_create(m, n, row_ptr, col, windows=windows)


@pytest.mark.parametrize("case", [
    "bad_row_ptr", "col_out_of_range", "dup_in_row", "overlap_too_big", "cn_uncovered",
    "cn_twice_in_group", "group_cn_range", "negative_overlap", "too_many_windows",
])
def test_create_rejects_malformed_input(nd, case):
    rp = [0, 2, 4, 6]
    col = [0, 1, 1, 2, 2, 3]
    m, n = 3, 4
    kw = {}
    if case == "bad_row_ptr":
        rp = [0, 3, 2, 6]
    elif case == "col_out_of_range":
        col = [0, 1, 1, 2, 2, 4]
    elif case == "dup_in_row":
        col = [0, 0, 1, 2, 2, 3]
    elif case == "overlap_too_big":
        kw = dict(windows=(1, 1, 1))
    elif case == "cn_uncovered":
        kw = dict(groups=[[0, 1]])
    elif case == "cn_twice_in_group":
        kw = dict(groups=[[0, 1, 1, 2]])
    elif case == "group_cn_range":
        kw = dict(groups=[[0, 1, 2, 3]])
    elif case == "negative_overlap":
        kw = dict(windows=(2, -1, 1))
    elif case == "too_many_windows":
        kw = dict(windows=(4, 0, 1))
    with pytest.raises(nd.LdpcError) as ei:
        _create(nd, m, n, rp, col, **kw)
    assert ei.value.code == nd.LDPC_EINVAL
    assert nd.ldpc_last_error()


def test_unsupported_sizes(nd):
    # n above 16-bit VN ids, and a CN of degree 33
    with pytest.raises(nd.LdpcError) as ei:
        _create(nd, 1, 70000, [0, 2], [0, 69999])
    assert ei.value.code == nd.LDPC_EUNSUPPORTED
    with pytest.raises(nd.LdpcError) as ei:
        _create(nd, 1, 40, [0, 33], list(range(33)))
    assert ei.value.code == nd.LDPC_EUNSUPPORTED


def test_decode_rejects_null_code(nd):
    with pytest.raises(nd.LdpcError) as ei:
        nd.ldpc_decode(0, 0, 1, 10, 0, 0, 0, 0, 0, 0)
    assert ei.value.code == nd.LDPC_EINVAL


def test_tune_rejects_null_code(nd):
    with pytest.raises(nd.LdpcError) as ei:
        nd.ldpc_code_tune(0, 0, 1)
    assert ei.value.code == nd.LDPC_EINVAL


def test_batch_argument_errors(nd):
    """Argument checks of the batch entry points that run before any HIP
    call; an empty batch needs no device at all."""
    import ctypes
    from paper_1202_1060_amd import _native
    lib = _native.load()
    out = ctypes.c_void_p()
    assert lib.ldpc_batch_create(None, 0, 0, None, None) == nd.LDPC_EINVAL
    assert lib.ldpc_batch_create(None, -1, 0, None, ctypes.byref(out)) == nd.LDPC_EINVAL
    assert lib.ldpc_batch_create(None, 1, 0, None, ctypes.byref(out)) == nd.LDPC_EINVAL
    assert lib.ldpc_batch_create(None, 0, 0x100, None, ctypes.byref(out)) == nd.LDPC_EINVAL
    assert lib.ldpc_batch_create(None, 0, nd.LDPC_FLAG_MSG_FP16 | nd.LDPC_FLAG_MSG_BF16, None,
                                 ctypes.byref(out)) == nd.LDPC_EINVAL
    for bad in ((3, 1, 0, 4), (0, 1, 100, 4), (0, 1, 2048, 4), (0, 1, 0, 9), (0, 1, 0, -1)):
        opt = _native.ldpc_batch_options(*bad)
        assert lib.ldpc_batch_create(None, 0, 0, ctypes.byref(opt), ctypes.byref(out)) == nd.LDPC_EINVAL, bad
    probs = (_native.ldpc_problem * 1)()
    probs[0].code = None
    probs[0].num_frames = 4
    probs[0].max_iter = 10
    assert lib.ldpc_batch_create(probs, 1, 0, None, ctypes.byref(out)) == nd.LDPC_EINVAL
    assert "code is NULL" in nd.ldpc_last_error()
    assert lib.ldpc_batch_create(None, 0, 0, None, ctypes.byref(out)) == nd.LDPC_OK
    info = _native.ldpc_batch_info()
    assert lib.ldpc_batch_query(out, ctypes.byref(info)) == nd.LDPC_OK
    assert (info.num_launches, info.num_problems, info.total_frames) == (0, 0, 0)
    assert lib.ldpc_batch_launch(out, None) == nd.LDPC_OK
    assert lib.ldpc_batch_destroy(out) == nd.LDPC_OK
    assert lib.ldpc_batch_launch(None, None) == nd.LDPC_EINVAL
    assert lib.ldpc_batch_destroy(None) == nd.LDPC_OK
    assert lib.ldpc_decode_batched(None, 0, 0, None) == nd.LDPC_OK


def test_destroy_null_is_ok(nd):
    from paper_1202_1060_amd import _native
    assert _native.load().ldpc_code_destroy(None) == 0


def test_regrouping_argument_checks(nd):
    """groups_per_iteration: explicit groups only, a divisor of num_groups,
    every CN covered by every block (checked before any device work)."""
    m, n = 4, 8
    rp, ci = [0, 2, 4, 6, 8], [0, 1, 2, 3, 4, 5, 6, 7]
    with pytest.raises(nd.LdpcError) as ei:   # 3 groups, 2 per iteration
        nd.ldpc_code_create(m, n, rp, ci, groups=[[0, 1], [2, 3], [0, 1, 2, 3]], groups_per_iteration=2)
    assert ei.value.code == nd.LDPC_EINVAL
    with pytest.raises(nd.LdpcError) as ei:   # block 1 misses CN 3
        nd.ldpc_code_create(m, n, rp, ci, groups=[[0, 1], [2, 3], [0, 1], [2]], groups_per_iteration=2)
    assert ei.value.code == nd.LDPC_EINVAL
    assert "block 1" in nd.ldpc_last_error()


@pytest.mark.parametrize("vn_groups,what", [
    ([[0, 1], [1, 2, 3]], "two groups"),
    ([[0, 1], [2]], "no group"),
    ([[0, 1], [2, 4]], "out of range"),
    ([[0, 1], []], "empty group"),
])
def test_vertical_grouping_argument_checks(nd, vn_groups, what):
    """VN groups (the vertical schedule) must partition the VNs; they are
    checked before any device work."""
    rp, col = [0, 2, 4, 6], [0, 1, 1, 2, 2, 3]
    with pytest.raises(nd.LdpcError) as ei:
        nd.ldpc_code_create(3, 4, rp, col, vn_groups=vn_groups)
    assert ei.value.code == nd.LDPC_EINVAL
    assert what in nd.ldpc_last_error()
    with pytest.raises(nd.LdpcError) as ei:
        nd.ldpc_code_create(3, 4, rp, col, vn_groups=[[0, 1], [2, 3]], groups_per_iteration=1)
    assert ei.value.code == nd.LDPC_EINVAL
