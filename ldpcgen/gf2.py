"""GF(2) linear algebra on bit-packed rows: rank and a systematic encoder.

The encoder brings H to reduced row-echelon form over GF(2) (Gauss-Jordan
on 64-bit packed rows). Pivot columns carry parity bits, the remaining
K = n - rank(H) columns carry the information bits, so every output word
satisfies c H^T = 0.
"""
from __future__ import annotations

import numpy as np


def _pack_rows(h: np.ndarray) -> np.ndarray:
    m, n = h.shape
    w = (n + 63) // 64
    padded = np.zeros((m, w * 64), dtype=np.uint8)
    padded[:, :n] = h
    bits = padded.reshape(m, w, 64)
    weights = (np.uint64(1) << np.arange(64, dtype=np.uint64))
    return (bits.astype(np.uint64) * weights).sum(axis=2, dtype=np.uint64)


def _rref(packed: np.ndarray, n: int):
    """In-place Gauss-Jordan elimination; returns the pivot columns."""
    m = packed.shape[0]
    pivots = []
    r = 0
    for c in range(n):
        if r == m:
            break
        w, b = divmod(c, 64)
        colbits = (packed[:, w] >> np.uint64(b)) & np.uint64(1)
        cand = np.nonzero(colbits[r:])[0]
        if cand.size == 0:
            continue
        p = r + int(cand[0])
        if p != r:
            packed[[r, p]] = packed[[p, r]]
        colbits = (packed[:, w] >> np.uint64(b)) & np.uint64(1)
        colbits[r] = 0
        rows = np.nonzero(colbits)[0]
        if rows.size:
            packed[rows] ^= packed[r]
        pivots.append(c)
        r += 1
    return pivots


def _unpack_rows(packed: np.ndarray, n: int) -> np.ndarray:
    m, w = packed.shape
    shifts = np.arange(64, dtype=np.uint64)
    bits = ((packed[:, :, None] >> shifts) & np.uint64(1)).astype(np.uint8)
    return bits.reshape(m, w * 64)[:, :n]


def gf2_rank(h: np.ndarray) -> int:
    h = np.asarray(h, dtype=np.uint8)
    return len(_rref(_pack_rows(h), h.shape[1]))


class SystematicEncoder:
    """Encoder for the code with parity-check matrix ``code`` (an
    :class:`ldpcgen.codes.Code`)."""

    def __init__(self, code):
        h = code.dense()
        self.n = code.n
        packed = _pack_rows(h)
        self.pivots = np.array(_rref(packed, code.n), dtype=np.int64)
        self.rank = len(self.pivots)
        self.k = code.n - self.rank
        is_piv = np.zeros(code.n, dtype=bool)
        is_piv[self.pivots] = True
        self.info_pos = np.nonzero(~is_piv)[0]
        rref = _unpack_rows(packed[: self.rank], code.n)
        # parity bit of pivot row i = sum_k A[i, k] u_k (mod 2)
        self.A = rref[:, self.info_pos].astype(np.float32)

    @property
    def rate(self) -> float:
        return self.k / self.n

    def encode(self, u: np.ndarray) -> np.ndarray:
        """u: (F, K) bits -> (F, n) codewords (uint8)."""
        u = np.asarray(u, dtype=np.uint8)
        f = u.shape[0]
        c = np.zeros((f, self.n), dtype=np.uint8)
        c[:, self.info_pos] = u
        if self.rank:
            par = u.astype(np.float32) @ self.A.T  # exact integers < 2^24
            c[:, self.pivots] = (par.astype(np.int64) & 1).astype(np.uint8)
        return c
