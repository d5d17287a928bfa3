"""ldpc_decode_noalloc (fixed per-GPU scratch, no allocation) against
ldpc_decode: the same kernels on the same inputs, so the outputs must be
equal bit for bit, in the LDS tier and in the HBM tier (where the scratch
bounds the tiles in flight), on two calls in a row, the second smaller;
a code whose HBM-tier tile exceeds the scratch is refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - needs a GPU
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1202_1060_amd as nd  # noqa: E402
from paper_1202_1060_amd import _native  # noqa: E402
from ldpcgen import workloads as W, regular_code, make_frames  # noqa: E402

DEV = torch.device("cuda:0")


def _run(fn, dcode, x, max_iter, flags):
    F = x.shape[0]
    out = nd.new_outputs(F, dcode.n, DEV, packed=bool(flags & nd.LDPC_FLAG_OUT_PACKED))
    fn(dcode.handle, x.data_ptr(), F, max_iter, flags, out["hard"].data_ptr(), out["post"].data_ptr(),
       out["iters"].data_ptr(), out["syn_ok"].data_ptr(), torch.cuda.current_stream().cuda_stream)
    return out


@pytest.mark.parametrize("msg,hbm", [("fp32", False), ("fp16", False), ("fp32", True), ("fp16", True)])
def test_noalloc_equals_decode(msg, hbm):
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    dcode = nd.Code(code, windows=rec["windows"])
    try:
        lo, _ = W.frames(rec, 1, num_frames=3000 if hbm else 5000, first_frame=11)
        x = torch.from_numpy(lo).to(DEV)
        flags = nd.msg_flag(msg) | nd.LDPC_FLAG_EARLY_STOP | (_native.LDPC_FLAG_TIER_HBM if hbm else 0)
        for F in (x.shape[0], 777):  # second call smaller
            want = _run(nd.ldpc_decode, dcode, x[:F], rec["max_iter"], flags)
            got = _run(nd.ldpc_decode_noalloc, dcode, x[:F], rec["max_iter"], flags)
            torch.cuda.synchronize()
            for k in want:
                assert torch.equal(got[k], want[k]), (msg, hbm, F, k)
    finally:
        dcode.close()


def test_noalloc_packed_and_fixed_iterations():
    code = W.code_n96()
    dcode = nd.Code(code, windows=(4, 2, 1))
    try:
        llr, _ = make_frames(code.n, 300, 2.0, 0.5, seed=71)
        x = torch.from_numpy(llr).to(DEV)
        for flags, F in ((nd.LDPC_FLAG_OUT_PACKED, 300), (nd.LDPC_FLAG_OUT_PACKED | nd.LDPC_FLAG_EARLY_STOP, 41)):
            want = _run(nd.ldpc_decode, dcode, x[:F], 10, flags)
            got = _run(nd.ldpc_decode_noalloc, dcode, x[:F], 10, flags)
            torch.cuda.synchronize()
            for k in want:
                assert torch.equal(got[k], want[k]), (flags, F, k)
    finally:
        dcode.close()


def test_noalloc_refuses_a_tile_beyond_the_scratch():
    """n = 65000 with four edges per VN: one 64-frame HBM tile of FP32
    messages needs about 83 MB, more than the 64 MiB scratch; nothing is
    launched. Arguments are checked as in ldpc_decode."""
    big = regular_code(65000, 4, 32, seed=5, girth6=False)
    dcode = nd.Code(big, windows=(4, 16, 1))
    try:
        x = torch.zeros((2, big.n), dtype=torch.float32, device=DEV)
        with pytest.raises(nd.LdpcError) as ei:
            _run(nd.ldpc_decode_noalloc, dcode, x, 5, nd.LDPC_FLAG_EARLY_STOP)
        assert ei.value.code == nd.LDPC_EUNSUPPORTED
        assert "scratch" in nd.ldpc_last_error()
        with pytest.raises(nd.LdpcError) as ei:
            _run(nd.ldpc_decode_noalloc, dcode, x, 0, 0)
        assert ei.value.code == nd.LDPC_EINVAL
    finally:
        dcode.close()
