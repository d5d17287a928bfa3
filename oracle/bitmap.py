"""Brute-force bitwise MAP LLRs over every codeword of a tiny code.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For channel LLRs L_j = ln p(y_j|0)/p(y_j|1) the codeword likelihood is
proportional to exp(sum_j (1 - 2c_j) L_j / 2), so the bitwise MAP LLR is
  ln sum_{c in C, c_n = 0} exp(.) - ln sum_{c in C, c_n = 1} exp(.).
On a cycle-free Tanner graph sum-product BP reaches these values exactly
once every message has crossed the graph.
"""
from __future__ import annotations

import itertools

import numpy as np


def codewords(h: np.ndarray) -> np.ndarray:
    """All words c with c H^T = 0 (enumerates 2^n words; n <= 22)."""
    h = np.asarray(h, dtype=np.int64)
    m, n = h.shape
    assert n <= 22
    words = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.int64)
    syn = (words @ h.T) % 2
    return words[np.all(syn == 0, axis=1)]


def map_llr(h: np.ndarray, llr) -> np.ndarray:
    llr = np.asarray(llr, dtype=np.float64)
    cw = codewords(h)
    metric = ((1 - 2 * cw) * llr[None, :]).sum(axis=1) / 2.0
    out = np.empty(len(llr))
    for j in range(len(llr)):
        a = metric[cw[:, j] == 0]
        b = metric[cw[:, j] == 1]
        out[j] = np.logaddexp.reduce(a) - np.logaddexp.reduce(b)
    return out
