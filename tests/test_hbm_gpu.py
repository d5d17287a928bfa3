"""HBM tier of the decoder (frame-interleaved state in device memory).

On a code that fits in LDS, the HBM tier (forced with LDPC_FLAG_TIER_HBM)
must equal the LDS tier with one lane per CN visit bit for bit: both run
cn_core on the same values in the same order. On a code beyond LDS it must
meet the oracle bar.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - needs a GPU
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1202_1060_amd as nd  # noqa: E402
from paper_1202_1060_amd import _native  # noqa: E402
from ldpcgen import workloads as W, make_frames  # noqa: E402
from ldpcgen.codes import qc_code, base_mask  # noqa: E402

from parity import compare, syndrome_zero  # noqa: E402

DEV = torch.device("cuda:0")


def _decode(dcode, llr, max_iter, early_stop, msg, hbm, packed=False, stream=None):
    x = torch.from_numpy(np.ascontiguousarray(llr, dtype=np.float32)).to(DEV)
    F = x.shape[0]
    out = nd.new_outputs(F, dcode.n, DEV, packed=packed)
    flags = (nd.msg_flag(msg) | (nd.LDPC_FLAG_EARLY_STOP if early_stop else 0)
             | (nd.LDPC_FLAG_OUT_PACKED if packed else 0) | (_native.LDPC_FLAG_TIER_HBM if hbm else 0))
    s = stream or torch.cuda.current_stream()
    nd.ldpc_decode(dcode.handle, x.data_ptr(), F, max_iter, flags, out["hard"].data_ptr(),
                   out["post"].data_ptr(), out["iters"].data_ptr(), out["syn_ok"].data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.fixture(scope="module")
def sweep():
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    lo, _ = W.frames(rec, 0, num_frames=150, first_frame=7)
    hi, _ = W.frames(rec, 4, num_frames=150, first_frame=7)
    llr = np.concatenate([lo, hi])  # 300 frames: 4 full tiles and a ragged one
    dcode = nd.Code(code, windows=rec["windows"])
    yield code, dcode, llr
    dcode.close()


@pytest.mark.parametrize("msg", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("early_stop", [True, False])
def test_hbm_tier_equals_lds_tier_one_lane(sweep, msg, early_stop):
    code, dcode, llr = sweep
    dcode.tune(msg, 1)
    try:
        want = _decode(dcode, llr, 20, early_stop, msg, hbm=False)
        got = _decode(dcode, llr, 20, early_stop, msg, hbm=True)
    finally:
        dcode.tune(msg, 0)
    for k in want:
        assert np.array_equal(got[k], want[k]), k
    assert np.array_equal(got["syn_ok"].astype(bool), syndrome_zero(code, got["hard"]))
    print(msg, early_stop, "decoded", got["syn_ok"].mean(), "mean iters", got["iters"].mean())


def test_hbm_tier_small_counts_packed_and_repeats(sweep):
    code, dcode, llr = sweep
    dcode.tune("fp16", 1)
    try:
        for F in (1, 63, 64, 65):
            want = _decode(dcode, llr[:F], 20, True, "fp16", hbm=False, packed=True)
            got = _decode(dcode, llr[:F], 20, True, "fp16", hbm=True, packed=True)
            for k in want:
                assert np.array_equal(got[k], want[k]), (F, k)
        # back-to-back HBM-tier launches on two streams share the workspace:
        # the library orders them on the device
        s2 = torch.cuda.Stream()
        x = torch.from_numpy(llr).to(DEV)
        outs = []
        for i in range(6):
            s = torch.cuda.current_stream() if i % 2 == 0 else s2
            o = nd.new_outputs(len(llr), code.n, DEV)
            nd.ldpc_decode(dcode.handle, x.data_ptr(), len(llr), 20,
                           nd.LDPC_FLAG_MSG_FP16 | nd.LDPC_FLAG_EARLY_STOP | _native.LDPC_FLAG_TIER_HBM,
                           o["hard"].data_ptr(), o["post"].data_ptr(), o["iters"].data_ptr(),
                           o["syn_ok"].data_ptr(), s.cuda_stream)
            outs.append(o)
        torch.cuda.synchronize()
        ref = _decode(dcode, llr, 20, True, "fp16", hbm=False)
        for o in outs:
            for k in ref:
                assert np.array_equal(o[k].cpu().numpy(), ref[k]), k
    finally:
        dcode.tune("fp16", 0)


@pytest.fixture(scope="module")
def big():
    # QC rate 1/2, z = 704, n = 16896: beyond LDS in every message format
    code = qc_code(base_mask("1/2", 1030), 704, 1030)
    dcode = nd.Code(code, windows=(12, 176, 1))
    yield code, dcode
    dcode.close()


def test_code_beyond_lds_meets_oracle_bar(big):
    code, dcode = big
    info = dcode.info
    assert info["lds_bytes_16"] > info["lds_limit"] and info["lds_bytes_fp32"] > info["lds_limit"]
    llr, _ = make_frames(code.n, 80, 1.6, 0.5, seed=1031)  # all-zero codeword
    got = _decode(dcode, llr, 15, True, "fp32", hbm=False)  # takes the HBM tier by itself
    groups = oracle.windows(code.m, 12, 176, True)
    ref = oracle.decode_with_sensitivity(code, groups, llr, 15, True)
    print("n=16896 fp32", compare(got, ref))
    g16 = _decode(dcode, llr, 15, True, "fp16", hbm=False)
    ok = ref["syn_ok"].astype(bool)
    assert np.mean(g16["hard"][ok] != ref["hard"][ok]) < 1e-3
    assert np.array_equal(g16["syn_ok"].astype(bool), syndrome_zero(code, g16["hard"]))


def test_batches_refuse_codes_beyond_lds(big):
    code, dcode = big
    x = torch.zeros((4, code.n), dtype=torch.float32, device=DEV)
    with pytest.raises(nd.LdpcError) as ei:
        nd.decode_batched([nd.Problem(dcode, x, 10)], msg="fp16")
    assert ei.value.code == nd.LDPC_EUNSUPPORTED


@pytest.mark.parametrize("msg", ["fp32", "fp16"])
def test_hbm_tier_degree_ten(msg):
    """Degree-10 variant (checks of degree 9 and 10): the HBM tier equals
    the one-lane LDS tier bit for bit."""
    code = W.CODES["qc1152r2_3"]()
    llr, _ = make_frames(code.n, 130, 2.4, 2 / 3, seed=93)
    dcode = nd.Code(code, windows=(9, 12, 1))
    try:
        dcode.tune(msg, 1)
        want = _decode(dcode, llr, 15, True, msg, hbm=False)
        got = _decode(dcode, llr, 15, True, msg, hbm=True)
    finally:
        dcode.close()
    for k in want:
        assert np.array_equal(got[k], want[k]), k
    print(msg, "decoded", got["syn_ok"].mean(), "mean iters", got["iters"].mean())
