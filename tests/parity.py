"""Shared helpers of the parity tests: run the HIP decoder and compare it with
the FP64 oracle.

Bar for FP32 messages, per frame, using the oracle's own conditioning
``sens`` (largest posterior change of the FP64 decode when every input LLR
moves by one float32 ulp; see oracle.decode_with_sensitivity):

* well-conditioned frames (decoded by the oracle and sens < SENS_WELL):
  hard decisions, iteration
  count and syndrome flag identical; every posterior within
  ATOL + RTOL |ref| (1e-3 absolute near zero, 1e-4 relative);
* ill-conditioned frames: the posterior tolerance widens by K_SENS * sens,
  because FP32 rounding at every message update is amplified the way the
  one-ulp input change is; frames the oracle decodes must still give
  identical decisions, and wherever the decisions match the syndrome flag
  and iteration count must match too; on frames the oracle does not decode
  decision differences are counted and capped at 2% of those frames, not
  counting frames whose FP64 decisions themselves change under a one-ulp
  input change (such a chaotic frame may end decoded on the GPU, with its
  own flag and count).
Across all frames hard decisions must match on >= 99.99%, or every
mismatch must sit in an undecoded, ill-conditioned frame.
"""
from __future__ import annotations

import numpy as np

RTOL = 1e-4
ATOL = 1e-3
SENS_WELL = 1e-4
K_SENS = 16.0
MIN_FRAME_MATCH = 0.9999


def gpu_decode(dcode, llr_np, max_iter, early_stop, msg="fp32", device="cuda:0"):
    import torch
    import paper_1202_1060_amd as nd
    llr = torch.from_numpy(np.ascontiguousarray(llr_np, dtype=np.float32)).to(device)
    out = nd.decode(dcode, llr, max_iter, early_stop=early_stop, msg=msg)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def compare(gpu, ref, rtol=RTOL, atol=ATOL, k_sens=K_SENS):
    """``ref`` comes from oracle.decode_with_sensitivity. Returns stats;
    raises AssertionError when the bar is missed."""
    F = ref["hard"].shape[0]
    sens = ref.get("sens", np.zeros(F))
    well = (sens < SENS_WELL) & (ref["syn_ok"] == 1)
    conv = ref["syn_ok"] == 1
    match = np.all(gpu["hard"] == ref["hard"], axis=1)
    err = np.abs(gpu["post"].astype(np.float64) - ref["post"])
    widen = np.where(well, 0.0, k_sens * np.where(np.isfinite(sens), sens, np.inf))
    bound = atol + rtol * np.abs(ref["post"]) + widen[:, None]
    pok = np.all(err <= bound, axis=1)
    strict_pok = np.all(err <= atol + rtol * np.abs(ref["post"]), axis=1)
    stats = dict(frames=F, oracle_converged=int(conv.sum()), well_conditioned=int(well.sum()),
                 decision_mismatch=int((~match).sum()),
                 strict_post_miss=int((match & ~strict_pok).sum()),
                 strict_post_miss_well=int((match & well & ~strict_pok).sum()),
                 max_abs_err_well=float(err[well & match].max()) if (well & match).any() else 0.0,
                 max_abs_err=float(err[match].max()) if match.any() else 0.0)
    # well-conditioned frames: the bar as stated
    w = well
    assert np.all(match[w]), f"decisions differ on {int((~match & w).sum())} well-conditioned frames"
    assert np.array_equal(gpu["iters"][w], ref["iters"][w]), "iteration counts differ (well-conditioned)"
    assert np.all(strict_pok[w]), f"posteriors out of bound on {int((w & ~strict_pok).sum())} " \
                                  f"well-conditioned frames (max err {err[w].max()})"
    # decoded frames: same codeword; wherever the decisions match (every
    # decoded frame among them): same syndrome flag and iteration count
    assert np.all(match[conv]), f"decisions differ on {int((~match & conv).sum())} decoded frames"
    if "syn_ok" in gpu:
        assert np.array_equal(gpu["syn_ok"][match], ref["syn_ok"][match]), "syndrome flags differ"
    assert np.array_equal(gpu["iters"][match], ref["iters"][match]), "iteration counts differ"
    # posteriors of every frame with matching decisions, widened where ill-conditioned
    assert np.all(pok[match]), f"posteriors out of the widened bound on {int((match & ~pok).sum())} frames"
    # undecoded frames: a decision difference counts against the cap unless
    # the FP64 oracle's own decisions on that frame change under a one-ulp
    # input change (sens = inf): there the result is not determined at the
    # precision of the float32 input, and no float32 decoder can match it
    # (such a frame may even end decoded, its flag and count then differ)
    nc = ~conv
    chaotic = ~np.isfinite(sens)
    nc_mis = int((~match & nc & ~chaotic).sum())
    stats["undecoded_mismatch_chaotic"] = int((~match & nc & chaotic).sum())
    assert match.sum() >= MIN_FRAME_MATCH * F or nc_mis <= max(1, int(0.02 * nc.sum())), \
        f"decisions match on {int(match.sum())}/{F} frames ({nc_mis} undecoded, oracle-stable)"
    return stats


def syndrome_zero(code, hard):
    """Per frame: True iff the hard decisions satisfy every check of
    ``code`` (computed on the host from H, independent of both decoders)."""
    hard = np.asarray(hard, dtype=np.uint8)
    rp = np.asarray(code.row_ptr, dtype=np.int64)
    ci = np.asarray(code.col_idx, dtype=np.int64)
    bits = hard[:, ci]
    par = np.zeros((hard.shape[0], len(rp) - 1), dtype=np.uint8)
    nz = rp[1:] > rp[:-1]
    par[:, nz] = np.bitwise_xor.reduceat(bits, rp[:-1][nz], axis=1)
    return ~np.any(par, axis=1)
