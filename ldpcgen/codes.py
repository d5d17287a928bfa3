"""Seeded LDPC parity-check matrices (Sec. II-B: an M x N sparse binary H).

Two families, both returned as CSR with sorted, duplicate-free rows:

* ``regular_code``: a (dv, dc)-regular code from the configuration model
  (random matching of VN sockets to CN sockets), with parallel edges and,
  optionally, 4-cycles removed by VN-endpoint swaps that keep every degree.
* ``qc_code``: a quasi-cyclic code lifted from a binary base matrix by
  seeded circulant shifts, with 4-cycles in the lift avoided where the
  shift search finds a solution (s11 - s12 + s22 - s21 != 0 mod z).

All randomness comes from numpy's Philox generator seeded by the caller.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy import sparse


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence(seed)))


@dataclass
class Code:
    """A binary parity-check matrix H (m x n) in CSR form."""

    m: int
    n: int
    row_ptr: np.ndarray  # int32 [m+1]
    col_idx: np.ndarray  # int32 [nnz], each row sorted ascending
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def rows(self):
        for i in range(self.m):
            yield self.col_idx[self.row_ptr[i]:self.row_ptr[i + 1]]

    def row(self, i):
        return self.col_idx[self.row_ptr[i]:self.row_ptr[i + 1]]

    def cn_degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def vn_degrees(self) -> np.ndarray:
        return np.bincount(self.col_idx, minlength=self.n)

    def to_scipy(self) -> sparse.csr_matrix:
        data = np.ones(self.nnz, dtype=np.int32)
        return sparse.csr_matrix((data, self.col_idx, self.row_ptr), shape=(self.m, self.n))

    def dense(self) -> np.ndarray:
        h = np.zeros((self.m, self.n), dtype=np.uint8)
        for i in range(self.m):
            h[i, self.row(i)] = 1
        return h

    @staticmethod
    def from_rows(rows, n, meta=None) -> "Code":
        rows = [np.unique(np.asarray(r, dtype=np.int64)) for r in rows]
        lens = [len(r) for r in rows]
        row_ptr = np.zeros(len(rows) + 1, dtype=np.int32)
        row_ptr[1:] = np.cumsum(lens)
        col = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
        return Code(len(rows), int(n), row_ptr, col, dict(meta or {}))

    @staticmethod
    def from_dense(h, meta=None) -> "Code":
        h = np.asarray(h)
        return Code.from_rows([np.nonzero(r)[0] for r in h], h.shape[1], meta)


def count_4cycles(code: Code) -> int:
    """Number of CN pairs that share two or more VNs (each such pair closes
    at least one 4-cycle in the Tanner graph)."""
    b = code.to_scipy()
    c = (b @ b.T).tocoo()
    mask = (c.row < c.col) & (c.data >= 2)
    return int(mask.sum())


def _bad_edges(cn, vn, m, n, girth6, rng):
    """Edge indices to perturb: one edge per parallel-edge pair and one edge
    per CN pair that shares two or more VNs."""
    e = len(vn)
    key = cn.astype(np.int64) * n + vn
    order = np.argsort(key, kind="stable")
    ks = key[order]
    dup = np.nonzero(ks[1:] == ks[:-1])[0]
    bad = set(order[dup + 1].tolist())
    if girth6:
        b = sparse.csr_matrix((np.ones(e, np.int32), (cn, vn)), shape=(m, n))
        b.data[:] = 1
        c = (b @ b.T).tocoo()
        sel = (c.row < c.col) & (c.data >= 2)
        if np.any(sel):
            # map (cn, vn) -> one edge index
            first = {}
            for idx in order:
                first.setdefault(int(key[idx]), int(idx))
            rows_a = c.row[sel]
            rows_b = c.col[sel]
            bcsr = b.tocsr()
            for a, bb in zip(rows_a, rows_b):
                va = bcsr.indices[bcsr.indptr[a]:bcsr.indptr[a + 1]]
                vb = bcsr.indices[bcsr.indptr[bb]:bcsr.indptr[bb + 1]]
                shared = np.intersect1d(va, vb)
                row = int(a) if rng.integers(2) == 0 else int(bb)
                v = int(shared[rng.integers(len(shared))])
                bad.add(first[row * n + v])
    return np.array(sorted(bad), dtype=np.int64)


def regular_code(n: int, dv: int, dc: int, seed, girth6: bool = True,
                 max_rounds: int = 20000) -> Code:
    """(dv, dc)-regular H from the configuration model.

    Socket matching: VN sockets (each VN repeated dv times) are shuffled and
    laid against CN sockets (CN i owns sockets i*dc .. i*dc+dc-1). Offending
    edges (parallel edges; with ``girth6`` also one edge of every CN pair that
    shares >= 2 VNs) have their VN endpoint swapped with a uniformly chosen
    edge until none remain. Swaps keep all degrees."""
    if (n * dv) % dc:
        raise ValueError("n*dv must be divisible by dc")
    e = n * dv
    m = e // dc
    rng = _rng(seed)
    vn = np.repeat(np.arange(n, dtype=np.int64), dv)
    rng.shuffle(vn)
    cn = np.repeat(np.arange(m, dtype=np.int64), dc)
    for _ in range(max_rounds):
        bad = _bad_edges(cn, vn, m, n, girth6, rng)
        if bad.size == 0:
            break
        partners = rng.integers(0, e, size=bad.size)
        for b_, p_ in zip(bad, partners):
            vn[b_], vn[p_] = vn[p_], vn[b_]
    else:
        raise RuntimeError("configuration model did not converge")
    rows = [np.sort(vn[i * dc:(i + 1) * dc]) for i in range(m)]
    code = Code.from_rows(rows, n, dict(kind="regular", dv=dv, dc=dc, seed=seed, girth6=girth6))
    assert code.nnz == e
    return code


# Degree profiles for 24-column base matrices, one per rate. Each entry lists
# (column weight, number of columns) and (row weight, number of rows); totals
# of both sides agree. The rate-1/2 profile has VN degrees {2,3,6} and CN
# degrees {6,7}; the others are seeded choices of this project.
QC_PROFILES = {
    "1/2": dict(mb=12, cols=[(2, 11), (3, 8), (6, 5)], rows=[(7, 4), (6, 8)]),
    "2/3": dict(mb=8, cols=[(2, 8), (3, 12), (6, 4)], rows=[(10, 4), (9, 4)]),
    "3/4": dict(mb=6, cols=[(2, 6), (3, 14), (4, 4)], rows=[(12, 4), (11, 2)]),
    "5/6": dict(mb=4, cols=[(2, 6), (3, 18)], rows=[(17, 2), (16, 2)]),
}


def base_mask(rate: str, seed, nb: int = 24) -> np.ndarray:
    """Binary base matrix (mb x nb) with the degree profile of ``rate``.

    Columns are placed in a seeded random order, heaviest first; each takes
    the rows with the largest remaining capacity (ties broken at random).
    This greedy (Havel-Hakimi style) placement always succeeds for these
    graphical profiles."""
    prof = QC_PROFILES[rate]
    mb = prof["mb"]
    rng = _rng(seed)
    colw = np.concatenate([np.full(c, w) for w, c in prof["cols"]])
    roww = np.concatenate([np.full(c, w) for w, c in prof["rows"]])
    assert len(colw) == nb and colw.sum() == roww.sum() and len(roww) == mb
    for _attempt in range(1000):
        perm_r = rng.permutation(mb)
        cap = roww[perm_r].copy()
        colperm = rng.permutation(nb)
        order = colperm[np.argsort(-colw[colperm], kind="stable")]
        mask = np.zeros((mb, nb), dtype=np.uint8)
        ok = True
        for c in order:
            w = colw[c]
            key = cap + rng.random(mb) * 0.5
            rows = np.argsort(-key, kind="stable")[:w]
            if np.any(cap[rows] <= 0):
                ok = False
                break
            mask[perm_r[rows], c] = 1
            cap[rows] -= 1
        if ok and np.all(cap == 0):
            return mask
    raise RuntimeError("base mask construction failed")


def qc_code(mask: np.ndarray, z: int, seed, avoid4: bool = True, tries: int = 400) -> Code:
    """Lift a binary base matrix by z x z circulant permutations.

    Entry (r, c) with shift s connects CN r*z+i to VN c*z+((i+s) mod z).
    With ``avoid4`` the shifts are re-drawn for entries on violated
    2x2 sub-blocks (s11 - s12 + s22 - s21 == 0 mod z) until none remain or
    ``tries`` rounds pass; the number left is kept in ``meta['quads_4cycle']``."""
    mask = np.asarray(mask, dtype=np.uint8)
    mb, nb = mask.shape
    rng = _rng(seed)
    shifts = np.where(mask > 0, rng.integers(0, z, size=mask.shape), -1)
    nzr = [np.nonzero(mask[r])[0] for r in range(mb)]

    def violations():
        bad = []
        for r1 in range(mb):
            for r2 in range(r1 + 1, mb):
                common = np.intersect1d(nzr[r1], nzr[r2])
                if len(common) < 2:
                    continue
                d = (shifts[r1, common] - shifts[r2, common]) % z
                # a violated quad has equal differences on two columns
                order = np.argsort(d, kind="stable")
                ds = d[order]
                same = np.nonzero(ds[1:] == ds[:-1])[0]
                for s in same:
                    bad.append((r1, r2, int(common[order[s]]), int(common[order[s + 1]])))
        return bad

    left = 0
    if avoid4:
        for _ in range(tries):
            bad = violations()
            left = len(bad)
            if not bad:
                break
            for (r1, r2, c1, c2) in bad:
                rr = (r1, r2)[rng.integers(2)]
                cc = (c1, c2)[rng.integers(2)]
                shifts[rr, cc] = rng.integers(0, z)
        left = len(violations())
    rows = []
    for r in range(mb):
        for i in range(z):
            cols = [c * z + (i + shifts[r, c]) % z for c in nzr[r]]
            rows.append(cols)
    code = Code.from_rows(rows, nb * z, dict(kind="qc", z=z, mb=mb, nb=nb, seed=seed,
                                             quads_4cycle=left))
    code.meta["shifts"] = shifts
    return code
