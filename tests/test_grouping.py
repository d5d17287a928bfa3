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
