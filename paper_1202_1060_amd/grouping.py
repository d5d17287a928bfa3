"""Check-node groupings of the method (Sec. II-A, II-C Step 1), the CoCSG
measure of a grouping (Sec. I, II-A) and a Step-1 variant that makes its
free choices for a large CoCSG, and the equal-complexity iteration budget
of Sec. IV.

These run on the host and produce explicit groups for ``Code(...,
groups=...)``; the decoder itself is the same for every grouping.

Step 1 with G groups of N_G CNs and overlap ratio r: group 1 is N_G CNs drawn
at random from the pool U of CNs not yet in any group; group g >= 2 takes
round(r N_G) CNs at random from the CNs that group g-1 added (group 1 itself
for g = 2) and (1 - r) N_G new CNs from U. Readings where the text is silent
or loose:

* N_G: the overlap identity G N_G - (G - 1) N_G r = M gives
  N_G = M / (G - (G - 1) r); it is rounded up (the paper's example takes 34
  for 252 / 7.6 = 33.2);
* r N_G is rounded to the nearest integer, and the new CNs per group are
  N_G - round(r N_G);
* U loses every group's new CNs (the text states it for g >= 3 only);
* the last group takes every CN still in U, so that every CN is decoded; a
  group that finds U shorter than its share takes what is left.
"""
from __future__ import annotations

import math

import numpy as np


def group_size(M: int, G: int, r: float) -> int:
    """N_G from G N_G - (G - 1) N_G r = M, rounded up."""
    if G < 1 or not (0.0 <= r < 1.0):
        raise ValueError("need G >= 1 and 0 <= r < 1")
    return int(math.ceil(M / (G - (G - 1) * r) - 1e-9))


def step1_groups(M: int, G: int, r: float, rng, N_G: int | None = None):
    """Random non-disjoint grouping of CNs 0..M-1 (Step 1). ``rng`` is a
    numpy Generator (the method's random draws are an input). Returns a list
    of G integer arrays, in processing order."""
    if N_G is None:
        N_G = group_size(M, G, r)
    if N_G > M:
        raise ValueError("N_G > M")
    k_old = int(round(r * N_G))
    k_new = N_G - k_old
    pool = list(rng.permutation(M))  # U in a random order: draws pop from it
    groups = []
    first = [pool.pop() for _ in range(min(N_G, len(pool)))]
    groups.append(np.array(sorted(first), dtype=np.int32))
    added = first  # the CNs the previous group took from U
    for g in range(1, G):
        take = len(pool) if g == G - 1 else min(k_new, len(pool))
        new = [pool.pop() for _ in range(take)]
        src = np.array(added if g > 1 else groups[0], dtype=np.int64)
        old = rng.choice(src, size=min(k_old, len(src)), replace=False) if k_old and len(src) else []
        grp = np.array(sorted(set(int(x) for x in old) | set(new)), dtype=np.int32)
        groups.append(grp)
        added = new if new else list(src)
    return groups


def disjoint_random_groups(M: int, G: int, rng):
    """Conventional GSBP grouping: a random partition of the CNs into G
    groups of nearly equal size (r = 0)."""
    perm = rng.permutation(M)
    return [np.sort(part).astype(np.int32) for part in np.array_split(perm, G)]


def _vn_sets(code):
    """N(m) of every CN as a Python set (from the CSR arrays)."""
    rp, ci = np.asarray(code.row_ptr), np.asarray(code.col_idx)
    return [set(ci[rp[m]:rp[m + 1]].tolist()) for m in range(len(rp) - 1)]


def cocsg(code, groups):
    """Connectivity of consecutive subgraphs (CoCSG, Sec. I and II-A): for
    each pair of neighbouring groups, the number of VNs adjacent to both
    (|N(G_k) & N(G_{k-1})|, k = 2..G). Returns (ell, per_pair), ell being
    the mean over the pairs (0.0 for a single group)."""
    nbr = _vn_sets(code)
    vns = [set().union(*(nbr[int(c)] for c in g)) if len(g) else set() for g in groups]
    per = [len(vns[k] & vns[k - 1]) for k in range(1, len(groups))]
    return (float(np.mean(per)) if per else 0.0), per


def cocsg_groups(code, G: int, r: float, rng, N_G: int | None = None):
    """Step 1 with its free choices made for a large CoCSG (the open
    direction of Sec. V: overlap and group choices that use the code
    structure). As in Step 1, group 1 is N_G random CNs and group g >= 2
    takes round(r N_G) CNs drawn at random from the CNs the previous group
    added; its N_G - round(r N_G) new CNs, instead of random ones from U,
    are taken one at a time as the CN of U adding the most VNs of the
    previous group's subgraph not yet in group g's (ties: the random order
    of U). The last group takes every CN left in U. ``rng`` supplies the
    random draws; returns G integer arrays in processing order."""
    M = len(np.asarray(code.row_ptr)) - 1
    if N_G is None:
        N_G = group_size(M, G, r)
    if N_G > M:
        raise ValueError("N_G > M")
    nbr = _vn_sets(code)
    k_old = int(round(r * N_G))
    k_new = N_G - k_old
    order = [int(x) for x in rng.permutation(M)]  # U in a random order
    pool = set(order)
    first = order[-N_G:] if N_G else []
    for c in first:
        pool.discard(c)
    groups = [np.array(sorted(first), dtype=np.int32)]
    added = first
    for g in range(1, G):
        src = np.array(added if g > 1 else groups[0], dtype=np.int64)
        old = [int(x) for x in rng.choice(src, size=min(k_old, len(src)), replace=False)] \
            if k_old and len(src) else []
        prev_vns = set().union(*(nbr[c] for c in groups[g - 1].tolist())) if len(groups[g - 1]) else set()
        have = set().union(*(nbr[c] for c in old)) if old else set()
        new = []
        if g == G - 1:
            new = [c for c in order if c in pool]
        else:
            cand = [c for c in order if c in pool]
            for _ in range(min(k_new, len(cand))):
                best, best_gain = None, -1
                for c in cand:
                    gain = len((nbr[c] & prev_vns) - have)
                    if gain > best_gain:
                        best, best_gain = c, gain
                cand.remove(best)
                new.append(best)
                have |= nbr[best]
        for c in new:
            pool.discard(c)
        groups.append(np.array(sorted(set(old) | set(new)), dtype=np.int32))
        added = new if new else list(src)
    return groups


def equal_complexity_iterations(M: int, I_max: int, G: int, N_G: int, r: float) -> int:
    """Iterations NDGSBP may run for the CN-update count of I_max flooding
    (or disjoint group-shuffled) iterations: M I_max / (M + (G - 1) N_G r)
    (Sec. IV), rounded down."""
    return int(math.floor(M * I_max / (M + (G - 1) * N_G * r) + 1e-9))


__all__ = ["group_size", "step1_groups", "disjoint_random_groups", "equal_complexity_iterations", "cocsg",
           "cocsg_groups"]
