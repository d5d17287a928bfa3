"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each check is independent of the oracle's own code: printed example sets
(Sec. II-A, Fig. 1), exact MAP marginals on cycle-free graphs, textbook
special cases (one group = flooding SPA, zero overlap = layered GSBP),
closed forms of the CN update, and a high-SNR invariant.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import literal, bitmap
from ldpcgen import Code, regular_code, make_frames

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _fig1():
    with open(os.path.join(GOLD, "fig1_reach_sets.json")) as f:
        return json.load(f)


def _rows0(rows1):
    return [[v - 1 for v in r] for r in rows1]


# ---------------------------------------------------------------- Fig. 1 sets

@pytest.mark.parametrize("sched", ["bp", "gsbp", "ndgsbp"])
def test_fig1_reach_sets(sched):
    g = _fig1()
    rows = _rows0(g["graph_rows_1based"])
    s = g["schedules"][sched]
    groups = _rows0(s["groups_1based"])
    trace = []
    literal.run(rows, 8, groups, 1, literal.ReachAlgebra(), trace=trace)
    for e in s["expect"]:
        got = sorted(v + 1 for v in trace[e["after"] - 1][e["vn"] - 1])
        assert got == e["set"], (sched, e, got)


def _gauss_seidel_reach(rows, n, groups):
    """Negative control: CNs of a group updated one after another, each
    seeing its predecessors' VN updates (not the paper's schedule)."""
    cols = [[] for _ in range(n)]
    for m, r in enumerate(rows):
        for v in r:
            cols[v].append(m)
    lcv = {(m, v): frozenset() for m, r in enumerate(rows) for v in r}
    lvc = {(m, v): frozenset([v]) for m, r in enumerate(rows) for v in r}
    trace = []
    for grp in groups:
        for m in grp:
            for v in rows[m]:
                lcv[(m, v)] = frozenset().union(*[lvc[(m, u)] for u in rows[m] if u != v])
            for v in rows[m]:
                for mm in cols[v]:
                    lvc[(mm, v)] = frozenset([v]).union(*[lcv[(k, v)] for k in cols[v] if k != mm])
        trace.append({v: frozenset().union(*[lcv[(m, v)] for m in cols[v]]) for v in range(n)})
    return trace


def test_fig1_sets_reject_sequential_within_group():
    g = _fig1()
    rows = _rows0(g["graph_rows_1based"])
    s = g["schedules"]["ndgsbp"]
    trace = _gauss_seidel_reach(rows, 8, _rows0(s["groups_1based"]))
    mism = 0
    for e in s["expect"]:
        got = sorted(v + 1 for v in trace[e["after"] - 1][e["vn"] - 1])
        mism += got != e["set"]
    assert mism > 0


def test_fig1_grouping_is_windows():
    # (r, G, N_G) = (0.5, 3, 2) on M = 4: G*N_G - (G-1)*N_G*r = 6 - 2 = 4 = M,
    # and the printed groups are contiguous windows without wraparound.
    w = oracle.windows(4, 3, 1, wrap=False)
    assert [list(x) for x in w] == [[0, 1], [1, 2], [2, 3]]
    G, NG, r = 3, 2, 0.5
    assert G * NG - (G - 1) * NG * r == 4


def _check_wrapped_windows(w, M, G, o, length):
    """The wraparound grouping as the workloads state it: G windows of
    `length` CNs, consecutive windows (the last and the first included)
    sharing exactly o CNs, the shared CNs being the tail of one window and
    the head of the next, every CN covered, M + G*o CN updates in all."""
    assert len(w) == G
    assert all(len(x) == length for x in w)
    assert sum(len(x) for x in w) == M + G * o
    assert set(np.concatenate(w).tolist()) == set(range(M))
    for g in range(G):
        a, b = list(w[g]), list(w[(g + 1) % G])
        assert len(set(a) & set(b)) == o, (g, set(a) & set(b))
        assert a[len(a) - o:] == b[:o]
        assert len(set(a)) == len(a)


def test_wrapped_windows_of_the_small_workload():
    # n=96 (3,6) code, m=48: 4 windows of 14 CNs with a 2-CN overlap, wrap
    w = oracle.windows(48, 4, 2, wrap=True)
    _check_wrapped_windows(w, 48, 4, 2, 14)
    want = [list(range(0, 14)), list(range(12, 26)), list(range(24, 38)), list(range(36, 48)) + [0, 1]]
    assert [list(x) for x in w] == want


def test_wrapped_windows_of_the_sweep_workload():
    # n=2304 (3,6) code, m=1152: 8 windows of 160 CNs with a 16-CN overlap, wrap
    w = oracle.windows(1152, 8, 16, wrap=True)
    _check_wrapped_windows(w, 1152, 8, 16, 160)
    for g in range(7):
        assert list(w[g]) == list(range(144 * g, 144 * g + 160))
    assert list(w[7]) == list(range(1008, 1152)) + list(range(16))


def test_windows_uneven_split_by_hand():
    # M=10, G=3, overlap 1: starts floor(0)=0, floor(10/3)=3, floor(20/3)=6
    assert [list(x) for x in oracle.windows(10, 3, 1, wrap=True)] == \
        [[0, 1, 2, 3], [3, 4, 5, 6], [6, 7, 8, 9, 0]]
    # without wrap the last window stops at M (G-1 overlaps, as in Fig. 1)
    assert [list(x) for x in oracle.windows(10, 3, 1, wrap=False)] == \
        [[0, 1, 2, 3], [3, 4, 5, 6], [6, 7, 8, 9]]
    # zero overlap partitions the CNs (the disjoint GSBP baseline)
    assert [list(x) for x in oracle.windows(10, 3, 0, wrap=True)] == \
        [[0, 1, 2], [3, 4, 5], [6, 7, 8, 9]]
    # one window holding every CN (flooding)
    assert [list(x) for x in oracle.windows(10, 1, 0, wrap=True)] == [list(range(10))]
    with pytest.raises(ValueError):
        oracle.windows(10, 2, 6, wrap=True)


# ------------------------------------------------------------- MAP on trees

def _random_tree(rng, n_vn, max_dc=4):
    """Random cycle-free Tanner graph: CNs attach one existing VN plus
    fresh VNs until n_vn VNs exist."""
    rows = []
    nv = 1
    while nv < n_vn:
        k = int(rng.integers(1, min(max_dc, n_vn - nv + 1)))
        old = int(rng.integers(0, nv))
        rows.append([old] + list(range(nv, nv + k)))
        nv += k
    return rows


def _code_from_rows(rows, n):
    return Code.from_rows(rows, n)


@pytest.mark.parametrize("seed", range(6))
def test_c_oracle_equals_map_on_trees(seed):
    rng = np.random.default_rng(100 + seed)
    if seed == 0:
        rows = _rows0(_fig1()["graph_rows_1based"])
        n = 8
    else:
        n = int(rng.integers(8, 17))
        rows = _random_tree(rng, n)
    code = _code_from_rows(rows, n)
    h = code.dense()
    llr = rng.normal(1.0, 1.5, size=n).astype(np.float32)
    want = bitmap.map_llr(h, llr.astype(np.float64))
    m = code.m
    schedules = {
        "flooding": [np.arange(m)],
        "gsbp": [np.arange(0, m // 2), np.arange(m // 2, m)] if m >= 2 else [np.arange(m)],
        "ndgsbp": oracle.windows(m, max(1, min(3, m - 1)), 1, wrap=True) if m >= 3 else [np.arange(m)],
    }
    for name, groups in schedules.items():
        out = oracle.decode(code, groups, llr[None], max_iter=2 * n, early_stop=False, nthreads=1)
        np.testing.assert_allclose(out["post"][0], want, rtol=0, atol=1e-9, err_msg=name)


def test_literal_equals_map_on_fig1():
    rows = _rows0(_fig1()["graph_rows_1based"])
    code = _code_from_rows(rows, 8)
    rng = np.random.default_rng(7)
    llr = rng.normal(0.8, 1.2, size=8)
    want = bitmap.map_llr(code.dense(), llr)
    for groups in ([[0, 1, 2, 3]], [[0, 1], [2, 3]], [[0, 1], [1, 2], [2, 3]]):
        tot, _, _, _ = literal.run(rows, 8, groups, 6, literal.RealAlgebra(llr))
        np.testing.assert_allclose(tot, want, atol=1e-10)


# ------------------------------------------- C oracle vs literal (with cycles)

def _random_code(rng, n, m, dc_lo=3, dc_hi=6):
    rows = [sorted(rng.choice(n, size=int(rng.integers(dc_lo, dc_hi + 1)), replace=False))
            for _ in range(m)]
    return rows


@pytest.mark.parametrize("seed", range(5))
def test_c_oracle_matches_literal_schedule(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(16, 30))
    m = n // 2
    rows = _random_code(rng, n, m)
    code = _code_from_rows(rows, n)
    G = int(rng.integers(2, 5))
    o = int(rng.integers(1, 3))
    groups = oracle.windows(m, G, o, wrap=True)
    llr = rng.normal(0.6, 1.0, size=(3, n)).astype(np.float32)
    iters = 4
    out = oracle.decode(code, groups, llr, max_iter=iters, early_stop=False, nthreads=2)
    for f in range(3):
        tot, hard, _, ok = literal.run(rows, n, [list(g) for g in groups], iters,
                                       literal.RealAlgebra(llr[f].astype(np.float64)))
        np.testing.assert_allclose(out["post"][f], tot, rtol=1e-9, atol=1e-9)
        assert list(out["hard"][f]) == hard
        assert bool(out["syn_ok"][f]) == ok


def _rotated_windows(m, G, o, shift):
    return [np.sort((np.asarray(g) + shift) % m).astype(np.int32) for g in oracle.windows(m, G, o, wrap=True)]


@pytest.mark.parametrize("seed", range(4))
def test_c_oracle_matches_literal_regrouping(seed):
    """A new grouping every iteration (Step 4 returns to Step 1): the C
    oracle's schedule against the independent literal decoder."""
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(16, 30))
    m = n // 2
    rows = _random_code(rng, n, m)
    code = _code_from_rows(rows, n)
    G, o = int(rng.integers(2, 4)), 1
    sched = []
    for b in range(3):
        sched += _rotated_windows(m, G, o, int(rng.integers(0, m)))
    llr = rng.normal(0.6, 1.0, size=(3, n)).astype(np.float32)
    out = oracle.decode(code, sched, llr, max_iter=5, early_stop=False, nthreads=2, groups_per_iteration=G)
    for f in range(3):
        tot, hard, _, ok = literal.run(rows, n, [list(g) for g in sched], 5,
                                       literal.RealAlgebra(llr[f].astype(np.float64)), groups_per_iteration=G)
        np.testing.assert_allclose(out["post"][f], tot, rtol=1e-9, atol=1e-9)
        assert list(out["hard"][f]) == hard


def test_regrouping_reductions():
    """Repeating one grouping R times is that grouping; one iteration uses
    the first block only; different blocks change the result."""
    rng = np.random.default_rng(11)
    code = regular_code(96, 3, 6, seed=1000)
    llr, _ = make_frames(96, 8, 1.5, 0.5, seed=5)
    A = _rotated_windows(code.m, 4, 2, 0)
    B = _rotated_windows(code.m, 4, 2, 7)
    plain = oracle.decode(code, A, llr, 6, False)
    rep = oracle.decode(code, A + A + A, llr, 6, False, groups_per_iteration=4)
    assert np.array_equal(plain["post"], rep["post"])
    one = oracle.decode(code, A + B, llr, 1, False, groups_per_iteration=4)
    assert np.array_equal(one["post"], oracle.decode(code, A, llr, 1, False)["post"])
    two = oracle.decode(code, A + B, llr, 2, False, groups_per_iteration=4)
    assert not np.array_equal(two["post"], oracle.decode(code, A, llr, 2, False)["post"])
    assert rng is not None


# ------------------------------------------------------ textbook special cases

def _tanh_cn(x):
    """Textbook CN rule on a vector: out_i = 2 atanh(prod_{j != i} tanh(x_j/2))."""
    t = np.tanh(0.5 * np.asarray(x, dtype=np.float64))
    out = np.empty(len(t))
    for i in range(len(t)):
        out[i] = 2.0 * np.arctanh(np.prod(np.delete(t, i)))
    return out


def _textbook_flooding(h, llr, iters):
    """Two-phase flooding SPA on a dense H: all CNs, then all VNs."""
    m, n = h.shape
    mask = h.astype(bool)
    q = np.where(mask, llr[None, :], 0.0)  # VN->CN
    r = np.zeros((m, n))
    for _ in range(iters):
        for i in range(m):
            idx = np.nonzero(mask[i])[0]
            r[i, idx] = _tanh_cn(q[i, idx])
        tot = llr + r.sum(axis=0)
        q = np.where(mask, tot[None, :] - r, 0.0)
    return llr + r.sum(axis=0)


def _textbook_layered(h, llr, layers, iters):
    """Posterior-form layered decoding: per layer, T = P - R on the layer's
    edges, new R from T (all CNs of the layer at once), then P = L + sum R."""
    m, n = h.shape
    mask = h.astype(bool)
    r = np.zeros((m, n))
    p = llr.astype(np.float64).copy()
    for _ in range(iters):
        for layer in layers:
            t = {i: p[np.nonzero(mask[i])[0]] - r[i, np.nonzero(mask[i])[0]] for i in layer}
            for i in layer:
                idx = np.nonzero(mask[i])[0]
                r[i, idx] = _tanh_cn(t[i])
            p = llr + r.sum(axis=0)
    return p


@pytest.mark.parametrize("seed", range(3))
def test_one_group_is_flooding(seed):
    code = regular_code(48, 3, 6, seed=300 + seed, girth6=False)
    rng = np.random.default_rng(seed)
    llr = rng.normal(0.7, 1.0, size=code.n).astype(np.float32)
    out = oracle.decode(code, oracle.windows(code.m, 1, 0), llr[None], 5, False, 1)
    want = _textbook_flooding(code.dense(), llr.astype(np.float64), 5)
    np.testing.assert_allclose(out["post"][0], want, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("seed", range(3))
def test_zero_overlap_is_layered_gsbp(seed):
    code = regular_code(48, 3, 6, seed=310 + seed, girth6=False)
    rng = np.random.default_rng(seed + 10)
    llr = rng.normal(0.7, 1.0, size=code.n).astype(np.float32)
    groups = oracle.windows(code.m, 4, 0)
    out = oracle.decode(code, groups, llr[None], 4, False, 1)
    want = _textbook_layered(code.dense(), llr.astype(np.float64), [list(g) for g in groups], 4)
    np.testing.assert_allclose(out["post"][0], want, rtol=1e-9, atol=1e-9)


def test_overlap_changes_the_result():
    # the overlap schedule is not the disjoint one: same code, different output
    code = regular_code(48, 3, 6, seed=320, girth6=False)
    llr = np.random.default_rng(3).normal(0.5, 1.0, size=code.n).astype(np.float32)
    a = oracle.decode(code, oracle.windows(code.m, 4, 0), llr[None], 1, False, 1)["post"]
    b = oracle.decode(code, oracle.windows(code.m, 4, 3), llr[None], 1, False, 1)["post"]
    assert np.max(np.abs(a - b)) > 1e-3


# ------------------------------------------------------- CN update closed forms

def test_phi_closed_forms():
    # phi(x) = -ln tanh(x/2): phi(ln 3) = ln 2, and phi is an involution
    assert abs(oracle.phi(math.log(3.0)) - math.log(2.0)) < 1e-15
    for x in [1e-6, 1e-3, 0.1, 0.8813735870195430, 1.0, 5.0, 20.0, 29.9]:
        assert abs(oracle.phi(oracle.phi(x)) - x) <= 1e-12 * max(1.0, x)
        # phi(x) = -ln tanh(x/2) = 2 atanh(exp(-x)); each form where FP64 holds it well
        ref = -math.log(math.tanh(x / 2)) if x < 1.0 else 2 * math.atanh(math.exp(-x))
        assert abs(oracle.phi(x) - ref) <= 1e-13 * ref


def test_boxplus_closed_forms():
    rng = np.random.default_rng(11)
    # one input (a degree-2 check): the message is the other input
    for x in rng.normal(0, 5, size=20):
        assert abs(oracle.boxplus([x]) - x) <= 1e-12 * max(1.0, abs(x))
    # two inputs (degree 3): 2 atanh(tanh(a/2) tanh(b/2))
    for a, b in rng.normal(0, 3, size=(20, 2)):
        want = 2 * math.atanh(math.tanh(a / 2) * math.tanh(b / 2))
        assert abs(oracle.boxplus([a, b]) - want) <= 1e-10 * max(1.0, abs(want))
    # sign rule: product of signs, -0.0 counts as positive
    assert oracle.boxplus([-1.0, 2.0]) < 0
    assert oracle.boxplus([-1.0, -2.0]) > 0
    assert oracle.boxplus([-0.0, 2.0]) > 0
    # clamp: magnitudes stay in [phi(30), 30]
    # both inputs clamp to 30: phi(2 phi(30)) = 30 - ln 2 to first order in e^-30
    assert abs(oracle.boxplus([50.0, 60.0]) - (30.0 - math.log(2.0))) < 1e-9
    assert abs(oracle.boxplus([]) - 30.0) < 1e-9  # a degree-1 check forces its bit
    assert abs(oracle.boxplus([0.0, 3.0])) <= oracle.phi(30.0) * 1.0001


# ------------------------------------------------------------ invariants

def test_high_snr_all_zero_decodes_in_one_iteration():
    code = regular_code(2304, 3, 6, seed=1001)
    for ebn0, it_max in ((6.0, 3), (10.0, 1)):
        llr, cw = make_frames(code.n, 8, ebn0, 0.5, seed=77)
        out = oracle.decode(code, oracle.windows(code.m, 8, 16), llr, 20, True, 4)
        assert np.all(out["syn_ok"] == 1)
        assert np.all(out["iters"] <= it_max)
        assert np.all(out["hard"] == 0)


def test_early_stop_iteration_count_is_first_zero_syndrome():
    code = regular_code(96, 3, 6, seed=1000)
    llr, _ = make_frames(code.n, 40, 2.0, 0.5, seed=5)
    groups = oracle.windows(code.m, 4, 2)
    es = oracle.decode(code, groups, llr, 10, True, 2)
    for f in range(40):
        it = int(es["iters"][f])
        assert 1 <= it <= 10
        if es["syn_ok"][f]:
            # the same frame run for exactly `it` iterations without early stop
            # ends with the same decision, and one iteration fewer had not converged
            fx = oracle.decode(code, groups, llr[f:f + 1], it, False, 1)
            assert fx["syn_ok"][0] == 1
            assert np.array_equal(fx["hard"][0], es["hard"][f])
            if it > 1:
                fp = oracle.decode(code, groups, llr[f:f + 1], it - 1, False, 1)
                assert fp["syn_ok"][0] == 0


# --- vertical (VN-group) shuffled schedule, the prior art of Sec. I --------

@pytest.mark.parametrize("seed", range(3))
def test_vertical_one_group_is_flooding(seed):
    """One VN group holding every VN is flooding BP, bit for bit."""
    code = regular_code(96, 3, 6, seed=10 + seed, girth6=True)
    llr, _ = make_frames(code.n, 24, 1.5, 0.5, seed=70 + seed)
    a = oracle.decode_vertical(code, [np.arange(code.n)], llr, 8, False, nthreads=1)
    b = oracle.decode(code, [np.arange(code.m)], llr, 8, False, nthreads=1)
    assert np.array_equal(a["post"], b["post"])


def test_vertical_schedule_closed_form():
    """c1 = {v0, v1}, c2 = {v1, v2} with VN groups {v1} then {v0, v2}: in the
    first sub-iteration v1 takes L0 (through c1) and L2 (through c2) and
    sends L1 + L2 to c1 and L1 + L0 to c2; in the second, v0 and v2 take
    those, so after one iteration every posterior is L0 + L1 + L2 (flooding
    gives L0 + L1 at v0). A degree-2 check passes its other input through
    unchanged (phi is an involution)."""
    code = Code.from_rows([[0, 1], [1, 2]], 3)
    L = np.array([[0.7, -1.3, 2.1]], dtype=np.float32)
    Ld = L.astype(np.float64)[0]
    v = oracle.decode_vertical(code, [[1], [0, 2]], L, 1, False, nthreads=1)
    np.testing.assert_allclose(v["post"][0], [Ld.sum()] * 3, rtol=0, atol=1e-12)
    f = oracle.decode(code, [[0, 1]], L, 1, False, nthreads=1)
    np.testing.assert_allclose(f["post"][0], [Ld[0] + Ld[1], Ld.sum(), Ld[1] + Ld[2]], rtol=0, atol=1e-12)
    # the other order: {v0, v2} first sees only channel values
    w = oracle.decode_vertical(code, [[0, 2], [1]], L, 1, False, nthreads=1)
    np.testing.assert_allclose(w["post"][0], [Ld[0] + Ld[1], Ld.sum(), Ld[1] + Ld[2]], rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_vertical_equals_map_on_trees(seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(8, 17))
    code = _code_from_rows(_random_tree(rng, n), n)
    llr = rng.normal(1.0, 1.5, size=n).astype(np.float32)
    want = bitmap.map_llr(code.dense(), llr.astype(np.float64))
    perm = rng.permutation(n)
    for groups in ([perm[: n // 2], perm[n // 2:]], [[int(x)] for x in perm]):
        out = oracle.decode_vertical(code, groups, llr[None], max_iter=2 * n, early_stop=False, nthreads=1)
        np.testing.assert_allclose(out["post"][0], want, rtol=0, atol=1e-9)


def test_stop_margin_matches_its_definition():
    """The oracle's stop margin (a diagnostic of the parity bar) equals its
    definition evaluated on the oracle's posteriors after each iteration:
    the minimum over the iterations run of (zero syndrome: the smallest |P|
    of a VN in some check; otherwise: the largest, over failing checks, of
    the smallest |P| in the check)."""
    from ldpcgen import workloads as W
    code = W.code_n96()
    groups = oracle.windows(code.m, 4, 2, True)
    llr, _ = make_frames(code.n, 12, 1.5, 0.5, seed=88)
    r = oracle.decode(code, groups, llr, 10, True)
    rp, ci = np.asarray(code.row_ptr), np.asarray(code.col_idx)
    for f in range(12):
        want = np.inf
        for l in range(1, int(r["iters"][f]) + 1):
            P = oracle.decode(code, groups, llr[f:f + 1], l, False)["post"][0]
            low = np.array([np.abs(P[ci[rp[m]:rp[m + 1]]]).min() for m in range(code.m)])
            par = np.array([np.bitwise_xor.reduce((P[ci[rp[m]:rp[m + 1]]] < 0).astype(int)) for m in range(code.m)])
            here = low.min() if not par.any() else low[par == 1].max()
            want = min(want, here)
        assert r["margin"][f] == want, f
