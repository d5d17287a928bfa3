"""The parity bar itself (tests/parity.py), on synthetic results: it must
pass identical results and the excused chaotic cases, and fail each kind of
real mismatch."""
import numpy as np
import pytest

from parity import compare, compare16, U16


def _ref(F=200, n=16, seed=0):
    rng = np.random.default_rng(seed)
    post = rng.normal(4.0, 2.0, size=(F, n))
    post[:, 0] = np.abs(post[:, 0]) + 1.0
    hard = (post < 0).astype(np.uint8)
    syn = np.ones(F, np.uint8)
    syn[:20] = 0  # 20 frames the oracle does not decode
    iters = np.where(syn == 1, 5, 30).astype(np.int32)
    sens = np.full(F, 1e-6)
    return dict(post=post, hard=hard, iters=iters, syn_ok=syn, sens=sens)


def _gpu(ref):
    return dict(post=ref["post"].astype(np.float32).copy(), hard=ref["hard"].copy(),
                iters=ref["iters"].copy(), syn_ok=ref["syn_ok"].copy())


def test_identical_results_pass():
    ref = _ref()
    st = compare(_gpu(ref), ref)
    assert st["decision_mismatch"] == 0


def test_decoded_frame_decision_flip_fails():
    ref = _ref()
    g = _gpu(ref)
    g["hard"][50, 3] ^= 1
    with pytest.raises(AssertionError):
        compare(g, ref)


def test_decoded_frame_iteration_mismatch_fails():
    ref = _ref()
    g = _gpu(ref)
    g["iters"][60] += 1
    with pytest.raises(AssertionError):
        compare(g, ref)


def test_undecoded_frame_with_matching_decisions_must_keep_flag_and_count():
    ref = _ref()
    g = _gpu(ref)
    g["syn_ok"][5] = 1
    with pytest.raises(AssertionError):
        compare(g, ref)
    g = _gpu(ref)
    g["iters"][5] -= 1
    with pytest.raises(AssertionError):
        compare(g, ref)


def test_well_conditioned_posterior_out_of_bound_fails():
    ref = _ref()
    g = _gpu(ref)
    g["post"][70, 2] += 0.01 + 1e-4 * abs(ref["post"][70, 2])
    with pytest.raises(AssertionError):
        compare(g, ref)


def test_chaotic_undecoded_frame_may_end_decoded():
    """FP64 leaves the frame undecoded and its own decisions change under a
    one-ulp input change (sens = inf): the GPU may end elsewhere, even
    decoded, with another iteration count."""
    ref = _ref()
    ref["sens"][7] = np.inf
    g = _gpu(ref)
    g["hard"][7, 1:4] ^= 1
    g["syn_ok"][7] = 1
    g["iters"][7] = 29
    st = compare(g, ref)
    assert st["undecoded_mismatch_chaotic"] == 1


def test_stable_undecoded_mismatches_need_the_frame_fraction():
    """Undecoded frames whose FP64 decisions do not change under a one-ulp
    input change may differ only within 0.01% of the frames, rounded up to a
    whole frame; with pooled=True the fraction is left to the caller."""
    ref = _ref(F=20000)
    ref["syn_ok"][:2000] = 0
    ref["iters"][:2000] = 30
    g = _gpu(ref)
    g["hard"][0, 5] ^= 1  # 1 of 20000 frames
    g["hard"][1, 5] ^= 1  # 2 of 20000: 0.01%
    st = compare(g, ref)
    assert st["undecoded_mismatch_stable"] == 2
    g["hard"][2, 5] ^= 1  # 3 of 20000: above
    with pytest.raises(AssertionError):
        compare(g, ref)
    st = compare(g, ref, pooled=True)
    assert st["decision_mismatch"] == 3


def test_small_sample_allows_one_stable_mismatch():
    """Below 10000 frames 0.01% rounds up to one frame; chaotic frames do
    not count."""
    ref = _ref()
    g = _gpu(ref)
    g["hard"][3, 2] ^= 1
    compare(g, ref)
    g["hard"][4, 2] ^= 1
    with pytest.raises(AssertionError):
        compare(g, ref)
    ref["sens"][4] = np.inf
    compare(g, ref)


def test_sixteen_bit_bar():
    """compare16: passes results within K16 units, fails a decision flip on a
    decoded frame, an iteration difference on a frame both decode, and a
    posterior beyond the bound."""
    ref = _ref()
    g = _gpu(ref)
    g["post"] = (ref["post"] + 30 * U16 * (np.abs(ref["post"]) + 30)).astype(np.float32)
    st = compare16(g, ref)
    assert 25 < st["max_units"] < 35
    bad = _gpu(ref)
    bad["hard"][40, 1] ^= 1
    with pytest.raises(AssertionError):
        compare16(bad, ref)
    bad = _gpu(ref)
    bad["iters"][41] += 1
    with pytest.raises(AssertionError):
        compare16(bad, ref)
    bad = _gpu(ref)
    bad["post"][42, 0] += 70 * U16 * (abs(ref["post"][42, 0]) + 30)
    with pytest.raises(AssertionError):
        compare16(bad, ref)
    # frames the oracle leaves undecoded are not held to the bound
    bad = _gpu(ref)
    bad["post"][5, 0] += 100.0
    compare16(bad, ref)


def test_stop_moved_only_where_undetermined():
    """A frame may stop at another iteration (same decisions) only if the
    oracle's stop margin is below the posterior tolerance; its posteriors
    are then held to the oracle's result at the GPU's iteration count."""
    ref = _ref()
    ref["margin"] = np.full(200, 0.5)
    g = _gpu(ref)
    g["iters"][60] += 1
    with pytest.raises(AssertionError):
        compare(g, ref)  # stop determined (margin 0.5 nats)
    ref["margin"][60] = 2e-5
    with pytest.raises(AssertionError):
        compare(g, ref)  # undetermined, but no rerun to check the posteriors against
    ref["rerun"] = lambda idx, it: ref["post"][idx]
    st = compare(g, ref)
    assert st["stop_moved"] == 1 and st["stop_marginal"] == 1
    ref["rerun"] = lambda idx, it: ref["post"][idx] + 1.0
    with pytest.raises(AssertionError):
        compare(g, ref)  # posteriors at the moved stop out of bound
