"""Reduced-precision message storage (FP16 / BF16 messages, FP32 arithmetic):
frame error rate against the FP32 form, and posterior error against the
FP64 oracle, on the rate-1/2 QC code with 12 one-row windows of overlap 24."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - needs a GPU
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1202_1060_amd as nd  # noqa: E402
from ldpcgen import workloads as W  # noqa: E402
from scipy.stats import beta  # noqa: E402

from parity import gpu_decode  # noqa: E402


def clopper_pearson(k, n, alpha=0.05):
    lo = 0.0 if k == 0 else beta.ppf(alpha / 2, k, n - k + 1)
    hi = 1.0 if k == n else beta.ppf(1 - alpha / 2, k + 1, n - k)
    return lo, hi


@pytest.fixture(scope="module")
def qc():
    rec = W.PRECISION
    code = W.CODES[rec["code"]]()
    dcode = nd.Code(code, windows=rec["windows"])
    yield rec, code, dcode
    dcode.close()


@pytest.mark.parametrize("snr", [0, 1])
@pytest.mark.parametrize("msg", ["fp16", "bf16"])
def test_fer_within_fp32_confidence_interval(qc, snr, msg):
    rec, code, dcode = qc
    llr, cw = W.frames(rec, snr)  # all 65536 frames
    ref = gpu_decode(dcode, llr, rec["max_iter"], True, "fp32")
    low = gpu_decode(dcode, llr, rec["max_iter"], True, msg)
    err_ref = np.any(ref["hard"] != cw, axis=1)
    err_low = np.any(low["hard"] != cw, axis=1)
    n = len(cw)
    k32, k16 = int(err_ref.sum()), int(err_low.sum())
    lo, hi = clopper_pearson(k32, n)
    print(f"{msg} {rec['ebn0'][snr]} dB: FER fp32 {k32 / n:.5f} [{lo:.5f}, {hi:.5f}], {msg} {k16 / n:.5f}, "
          f"mean iters {ref['iters'].mean():.3f} / {low['iters'].mean():.3f}")
    assert lo <= k16 / n <= hi


@pytest.mark.parametrize("msg", ["fp16", "bf16"])
def test_posterior_error_against_oracle(qc, msg):
    """Reported, with a loose bound: the message rounding (2^-11 relative for
    FP16, 2^-8 for BF16) is propagated by every later update."""
    rec, code, dcode = qc
    llr, _ = W.frames(rec, 1, num_frames=96)
    g = gpu_decode(dcode, llr, rec["max_iter"], True, msg)
    r = oracle.decode(code, oracle.windows(code.m, *rec["windows"][:2], True), llr, rec["max_iter"], True)
    conv = (r["syn_ok"] == 1) & (g["syn_ok"] == 1)
    rel = np.abs(g["post"][conv] - r["post"][conv]) / np.maximum(np.abs(r["post"][conv]), 1.0)
    same = np.all(g["hard"] == r["hard"], axis=1)
    print(f"{msg}: decoded by both {conv.sum()}/96, decisions equal {same.sum()}/96, "
          f"median rel err {np.median(rel):.2e}, max rel err {rel.max():.2e}")
    assert same[conv].all()
    assert np.median(rel) < (2e-3 if msg == "fp16" else 2e-2)
