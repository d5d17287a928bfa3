"""Step-1 grouping and the equal-complexity budget (host side, CPU only).

Pins: the paper's worked numbers for the (504,252) code with G = 12 and
r = 0.4 (N_G = 34, at most 627 iterations for I_max = 1000), the structure
Step 1 prescribes (group sizes, overlaps drawn from the previous group's new
CNs, every CN covered), and the two reductions (r = 0: disjoint; G = 1: one
group holding every CN).
"""
import numpy as np
import pytest

from paper_1202_1060_amd.grouping import (group_size, step1_groups, disjoint_random_groups,
                                          equal_complexity_iterations)


def _rng(s):
    return np.random.Generator(np.random.Philox(s))


def test_paper_example_numbers():
    # Sec. IV: G = 12, r = 0.4 on M = 252 gives N_G = 34 and ~627 iterations
    assert group_size(252, 12, 0.4) == 34
    assert equal_complexity_iterations(252, 1000, 12, 34, 0.4) == 627
    # Sec. II-A example (r, G, N_G) = (0.5, 3, 2) on 4 CNs
    assert group_size(4, 3, 0.5) == 2
    # no overlap: the budget is I_max itself
    assert equal_complexity_iterations(252, 1000, 12, 21, 0.0) == 1000


@pytest.mark.parametrize("M,G,r,seed", [(252, 12, 0.4, 1), (544, 16, 0.4, 2), (1152, 8, 0.25, 3),
                                        (4, 3, 0.5, 4), (100, 7, 0.3, 5)])
def test_step1_structure(M, G, r, seed):
    N_G = group_size(M, G, r)
    k_old = int(round(r * N_G))
    groups = step1_groups(M, G, r, _rng(seed), N_G)
    assert len(groups) == G
    allc = np.concatenate(groups)
    assert set(allc.tolist()) == set(range(M))  # every CN decoded
    for g in groups:
        assert len(np.unique(g)) == len(g)  # no CN twice in a group
    assert len(groups[0]) == N_G
    new_prev = set(groups[0].tolist())
    seen = set(groups[0].tolist())
    for g in range(1, G):
        cur = set(groups[g].tolist())
        old = cur & seen
        new = cur - seen
        # the overlap comes from the CNs the previous group added
        assert old <= new_prev, g
        assert len(old) == min(k_old, len(new_prev))
        if g < G - 1:
            assert len(new) == min(N_G - k_old, M - len(seen))
        seen |= new
        new_prev = new if new else new_prev
    # CN updates per iteration: M plus the overlaps
    assert sum(len(g) for g in groups) == M + sum(
        len(set(groups[g].tolist()) & set(np.concatenate(groups[:g]).tolist())) for g in range(1, G))


def test_fig1_example_shape():
    groups = step1_groups(4, 3, 0.5, _rng(9), 2)
    assert [len(g) for g in groups] == [2, 2, 2]
    assert len(set(groups[0]) & set(groups[1])) == 1 and len(set(groups[1]) & set(groups[2])) == 1
    assert not set(groups[0]) & set(groups[2])


def test_reductions():
    d = step1_groups(252, 12, 0.0, _rng(1))
    assert sorted(np.concatenate(d).tolist()) == list(range(252))  # a partition
    one = step1_groups(50, 1, 0.0, _rng(1))
    assert len(one) == 1 and sorted(one[0].tolist()) == list(range(50))
    part = disjoint_random_groups(252, 12, _rng(2))
    assert sorted(np.concatenate(part).tolist()) == list(range(252))
    assert {len(p) for p in part} == {21}


def test_step1_is_seeded():
    a = step1_groups(252, 12, 0.4, _rng(7))
    b = step1_groups(252, 12, 0.4, _rng(7))
    c = step1_groups(252, 12, 0.4, _rng(8))
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not all(np.array_equal(x, y) for x, y in zip(a, c))


# --- CoCSG (connectivity of consecutive subgraphs, Sec. I and II-A) --------

import json  # noqa: E402
import os  # noqa: E402

from ldpcgen import Code, regular_code  # noqa: E402
from paper_1202_1060_amd.grouping import cocsg, cocsg_groups  # noqa: E402


def _fig1():
    with open(os.path.join(os.path.dirname(__file__), "golden", "fig1_reach_sets.json")) as f:
        rows = json.load(f)["graph_rows_1based"]
    return Code.from_rows([[v - 1 for v in r] for r in rows], 8)


def test_cocsg_fig1_example():
    """On the Fig. 1 graph the non-disjoint grouping of the text shares more
    VNs between neighbouring groups than the disjoint one (the larger CoCSG
    that Sec. I claims): {c1,c2},{c3,c4} share v4 only; {c1,c2},{c2,c3}
    share v2, v4, v5 and {c2,c3},{c3,c4} share v4, v6, v7."""
    code = _fig1()
    ell_gs, per_gs = cocsg(code, [[0, 1], [2, 3]])
    ell_nd, per_nd = cocsg(code, [[0, 1], [1, 2], [2, 3]])
    assert per_gs == [1] and ell_gs == 1.0
    assert per_nd == [3, 3] and ell_nd == 3.0
    assert cocsg(code, [[0, 1, 2, 3]]) == (0.0, [])


def test_cocsg_brute_force():
    rng = np.random.default_rng(8)
    code = regular_code(60, 3, 6, seed=2, girth6=False)
    rows = [set(code.col_idx[code.row_ptr[m]:code.row_ptr[m + 1]].tolist()) for m in range(code.m)]
    for _ in range(5):
        groups = [rng.choice(code.m, size=int(rng.integers(1, 12)), replace=False) for _ in range(5)]
        want = []
        for k in range(1, 5):
            both = [v for v in range(code.n) if any(v in rows[c] for c in groups[k])
                    and any(v in rows[c] for c in groups[k - 1])]
            want.append(len(both))
        assert cocsg(code, groups)[1] == want


@pytest.mark.parametrize("key,G", [("n504", 12), ("n816", 16)])
def test_cocsg_bound_and_greedy_grouping(key, G):
    """The paper's relation ell >= (M/N) N_G r holds for Step-1 groupings and
    for the CoCSG-seeking variant, which keeps Step 1's structure and raises
    ell on average."""
    from ldpcgen import workloads as W
    code = W.CODES[key]()
    M, N, r = code.m, code.n, 0.4
    N_G = group_size(M, G, r)
    a, b = [], []
    for seed in range(4):
        g1 = step1_groups(M, G, r, _rng(100 + seed), N_G)
        g2 = cocsg_groups(code, G, r, _rng(100 + seed), N_G)
        for groups, acc in ((g1, a), (g2, b)):
            ell, per = cocsg(code, groups)
            assert ell >= M / N * N_G * r
            acc.append(ell)
        assert all(len(np.unique(g)) == len(g) for g in g2)  # no CN twice in a group
        assert set(np.concatenate(g2).tolist()) == set(range(M))
        assert [len(g) for g in g2[:-1]] == [len(g) for g in g1[:-1]]
        assert sum(len(g) for g in g2) == sum(len(g) for g in g1)  # same CN updates per iteration
    assert np.mean(b) > 1.1 * np.mean(a)


def test_cocsg_groups_structure():
    """The same structure Step 1 prescribes: group 1 of N_G CNs; each later
    group takes round(r N_G) of the previous group's new CNs plus new ones;
    every CN covered."""
    from ldpcgen import workloads as W
    code = W.CODES["n504"]()
    M, G, r = code.m, 12, 0.4
    N_G = group_size(M, G, r)
    k_old = int(round(r * N_G))
    groups = cocsg_groups(code, G, r, _rng(7), N_G)
    assert len(groups) == G and len(groups[0]) == N_G
    new_prev, seen = set(groups[0].tolist()), set(groups[0].tolist())
    for g in range(1, G):
        cur = set(groups[g].tolist())
        old, new = cur & seen, cur - seen
        assert old <= new_prev and len(old) == min(k_old, len(new_prev))
        if g < G - 1:
            assert len(new) == min(N_G - k_old, M - len(seen))
        seen |= new
        new_prev = new if new else new_prev
    assert seen == set(range(M))
