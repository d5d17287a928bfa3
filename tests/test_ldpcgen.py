"""Seeded input generators: codes, encoder, channel."""
import math

import numpy as np
import pytest

from ldpcgen import (regular_code, qc_code, base_mask, QC_PROFILES, count_4cycles,
                     SystematicEncoder, gf2_rank, ebn0_to_sigma, make_frames)
from ldpcgen import workloads as W


@pytest.mark.parametrize("n,seed", [(96, 1000), (2304, 1001)])
def test_regular_code_degrees_and_girth(n, seed):
    c = regular_code(n, 3, 6, seed=seed)
    assert c.m == n // 2 and c.nnz == 3 * n
    assert np.all(c.vn_degrees() == 3) and np.all(c.cn_degrees() == 6)
    assert count_4cycles(c) == 0
    for r in c.rows():
        assert len(np.unique(r)) == len(r)


def test_regular_code_is_seeded():
    a = regular_code(96, 3, 6, seed=5)
    b = regular_code(96, 3, 6, seed=5)
    c = regular_code(96, 3, 6, seed=6)
    assert np.array_equal(a.col_idx, b.col_idx)
    assert not np.array_equal(a.col_idx, c.col_idx)


@pytest.mark.parametrize("rate", list(QC_PROFILES))
def test_base_mask_profile(rate):
    prof = QC_PROFILES[rate]
    mask = base_mask(rate, seed=3)
    assert mask.shape == (prof["mb"], 24)
    want_c = sorted(np.concatenate([np.full(c, w) for w, c in prof["cols"]]))
    want_r = sorted(np.concatenate([np.full(c, w) for w, c in prof["rows"]]))
    assert sorted(mask.sum(axis=0)) == want_c
    assert sorted(mask.sum(axis=1)) == want_r


def test_qc_code_structure():
    c = W.CODES["qc2304"]()
    assert (c.m, c.n) == (1152, 2304)
    assert set(np.unique(c.vn_degrees())) == {2, 3, 6}
    assert set(np.unique(c.cn_degrees())) == {6, 7}
    assert c.meta["quads_4cycle"] == 0 and count_4cycles(c) == 0


def test_encoder_codewords_satisfy_checks():
    for key in ("n96", "n2304", "qc2304"):
        code = W.CODES[key]()
        enc = W.encoder_for(key)
        assert enc.rank == gf2_rank(code.dense())
        assert enc.k == code.n - enc.rank
        u = np.random.default_rng(0).integers(0, 2, size=(64, enc.k), dtype=np.uint8)
        cw = enc.encode(u)
        assert np.array_equal(cw[:, enc.info_pos], u)
        syn = (code.to_scipy() @ cw.T.astype(np.int64)) % 2
        assert not np.any(syn)


def test_sigma_convention():
    # sigma^2 = 1/(2 R Eb/N0): R = 1/2 at 0 dB gives sigma = 1; the (3,6)
    # GA threshold 1.163 dB quoted in Table I is sigma ~ 0.8747
    assert abs(ebn0_to_sigma(0.0, 0.5) - 1.0) < 1e-15
    assert abs(ebn0_to_sigma(1.163, 0.5) - 0.8747) < 2e-4


def test_frames_blocks_are_independent():
    code = W.code_n96()
    enc = W.encoder_for("n96")
    full, cw = make_frames(code.n, 600, 2.0, enc.rate, 9, encoder=enc)
    part, cwp = make_frames(code.n, 100, 2.0, enc.rate, 9, encoder=enc, first_frame=300)
    assert np.array_equal(full[300:400], part) and np.array_equal(cw[300:400], cwp)
    # LLR statistics: mean 2/sigma^2 * (1-2c), std 2/sigma
    s = ebn0_to_sigma(2.0, enc.rate)
    signed = full * (1 - 2 * cw.astype(np.float32))
    assert abs(signed.mean() - 2 / s**2) < 0.05 * 2 / s**2
    assert abs(signed.std() - 2 / s) < 0.05 * 2 / s
    assert full.dtype == np.float32
