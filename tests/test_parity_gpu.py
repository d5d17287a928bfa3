"""Parity of the HIP decoder (through the C ABI) with the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - needs a GPU
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1202_1060_amd as nd  # noqa: E402
from ldpcgen import Code, regular_code, make_frames  # noqa: E402
from ldpcgen import workloads as W  # noqa: E402

from parity import gpu_decode, compare, compare16  # noqa: E402


def _groups(code, windows):
    G, o, wrap = windows
    return oracle.windows(code.m, G, o, bool(wrap))


def _run_both(code, windows, llr, max_iter, early_stop, msg="fp32", nthreads=0, lanes=0):
    dcode = nd.Code(code, windows=windows)
    try:
        if lanes:
            dcode.tune(msg, lanes)
        g = gpu_decode(dcode, llr, max_iter, early_stop, msg)
    finally:
        dcode.close()
    r = oracle.decode_with_sensitivity(code, _groups(code, windows), llr, max_iter, early_stop, nthreads)
    return g, r


def test_small_workload():
    rec = W.SMALL
    code = W.CODES[rec["code"]]()
    llr, _ = W.frames(rec, 0)
    g, r = _run_both(code, rec["windows"], llr, rec["max_iter"], rec["early_stop"])
    st = compare(g, r)
    print("small", st)
    assert np.all(g["iters"] == rec["max_iter"])


@pytest.mark.parametrize("snr", range(7))
def test_sweep_early_stop(snr):
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    llr, _ = W.frames(rec, snr, num_frames=160)
    g, r = _run_both(code, rec["windows"], llr, rec["max_iter"], True)
    print("sweep", rec["ebn0"][snr], compare(g, r))


@pytest.mark.parametrize("snr", [0, 3])
def test_sweep_fixed_iterations(snr):
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    llr, _ = W.frames(rec, snr, num_frames=96, first_frame=1000)
    g, r = _run_both(code, rec["windows"], llr, rec["max_iter"], False)
    print("fixed", rec["ebn0"][snr], compare(g, r))
    assert np.all(g["iters"] == rec["max_iter"])


@pytest.mark.parametrize("recipe", ["flooding", "gsbp"])
def test_baseline_schedules(recipe):
    rec = W.SWEEP_FLOODING if recipe == "flooding" else W.SWEEP_GSBP
    code = W.CODES[rec["code"]]()
    llr, _ = W.frames(rec, 2, num_frames=128)
    g, r = _run_both(code, rec["windows"], llr, rec["max_iter"], True)
    print(recipe, compare(g, r))


def test_full_batch_sampled_frames():
    """All 16384 frames of one Eb/N0 point in one launch; the oracle checks
    a random sample of them."""
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    llr, _ = W.frames(rec, 2)
    dcode = nd.Code(code, windows=rec["windows"])
    g = gpu_decode(dcode, llr, rec["max_iter"], True)
    dcode.close()
    idx = np.sort(np.random.default_rng(1).choice(llr.shape[0], size=48, replace=False))
    r = oracle.decode_with_sensitivity(code, _groups(code, rec["windows"]), llr[idx], rec["max_iter"], True)
    print("sampled", compare({k: v[idx] for k, v in g.items()}, r))
    assert g["iters"].min() >= 1 and g["iters"].max() <= rec["max_iter"]


def test_qc_code_fp32():
    rec = W.PRECISION
    code = W.CODES[rec["code"]]()
    llr, _ = W.frames(rec, 0, num_frames=128)
    g, r = _run_both(code, rec["windows"], llr, rec["max_iter"], True)
    print("qc", compare(g, r))


def test_deterministic_bitwise():
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    llr, _ = W.frames(rec, 1, num_frames=256)
    dcode = nd.Code(code, windows=rec["windows"])
    a = gpu_decode(dcode, llr, rec["max_iter"], True)
    b = gpu_decode(dcode, llr, rec["max_iter"], True)
    dcode.close()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_unaligned_buffers_equal_aligned():
    """Buffers that are not 16-byte aligned (LLRs and posteriors 4 bytes
    past it, hard decisions 1 byte past) take the one-word frame start and
    output loops of the one-code kernel; the results equal those of aligned
    buffers (the 16-byte loops) bit for bit."""
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    llr, _ = W.frames(rec, 2, num_frames=300)
    F, n = llr.shape
    dcode = nd.Code(code, windows=rec["windows"])
    try:
        a = gpu_decode(dcode, llr, rec["max_iter"], True)
        dev = torch.device("cuda:0")
        lb = torch.zeros(F * n + 4, dtype=torch.float32, device=dev)
        x = lb[1:1 + F * n].view(F, n)
        x.copy_(torch.from_numpy(llr))
        hb = torch.zeros(F * n + 4, dtype=torch.uint8, device=dev)
        pb = torch.zeros(F * n + 4, dtype=torch.float32, device=dev)
        out = dict(hard=hb[1:1 + F * n].view(F, n), post=pb[1:1 + F * n].view(F, n),
                   iters=torch.empty(F, dtype=torch.int32, device=dev),
                   syn_ok=torch.empty(F, dtype=torch.uint8, device=dev))
        assert x.data_ptr() % 16 == 4 and out["hard"].data_ptr() % 4 == 1
        nd.decode(dcode, x, rec["max_iter"], early_stop=True, out=out)
        torch.cuda.synchronize()
        for k in a:
            assert np.array_equal(out[k].cpu().numpy(), a[k]), k
        # the bytes around the outputs are untouched
        assert int(hb[0]) == 0 and int(hb[-3:].sum()) == 0
        assert float(pb[0]) == 0.0 and float(pb[-3:].abs().sum()) == 0.0
    finally:
        dcode.close()


def test_explicit_groups_equal_windows():
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    llr, _ = W.frames(rec, 1, num_frames=64)
    a_code = nd.Code(code, windows=rec["windows"])
    b_code = nd.Code(code, groups=_groups(code, rec["windows"]))
    a = gpu_decode(a_code, llr, rec["max_iter"], True)
    b = gpu_decode(b_code, llr, rec["max_iter"], True)
    a_code.close()
    b_code.close()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("windows", [(5, 3, 1), (5, 3, 0), (7, 0, 1), (1, 0, 0), (48, 1, 1)])
def test_ragged_and_degenerate_windows(windows):
    """M=48 split unevenly, no wraparound, single-CN windows, one window."""
    code = W.code_n96()
    llr, _ = make_frames(code.n, 64, 1.5, 0.5, seed=31)
    g, r = _run_both(code, windows, llr, 8, True)
    print(windows, compare(g, r))


def test_low_and_high_degree_checks():
    """Degree-1 and degree-2 checks and a degree-20 check in one code."""
    rng = np.random.default_rng(4)
    n = 60
    rows = [[0], [1, 2], [3, 4]] + [sorted(rng.choice(n, size=int(rng.integers(3, 8)), replace=False))
                                     for _ in range(24)]
    rows.append(sorted(rng.choice(n, size=20, replace=False)))
    code = Code.from_rows(rows, n)
    llr, _ = make_frames(n, 64, 2.0, 0.5, seed=32)
    g, r = _run_both(code, (4, 2, 1), llr, 10, False)
    print("degrees", compare(g, r))


def test_tree_code_reaches_map():
    from oracle import bitmap
    rows = [[0, 1, 2], [1, 3, 4], [3, 5, 6], [6, 7]]
    code = Code.from_rows(rows, 8)
    rng = np.random.default_rng(9)
    llr = rng.normal(1.0, 1.5, size=(32, 8)).astype(np.float32)
    dcode = nd.Code(code, groups=[[0, 1], [1, 2], [2, 3]])
    g = gpu_decode(dcode, llr, 8, False)
    dcode.close()
    for f in range(32):
        want = bitmap.map_llr(code.dense(), llr[f].astype(np.float64))
        np.testing.assert_allclose(g["post"][f], want, rtol=1e-4, atol=1e-4)


def test_zero_and_one_frame():
    code = W.code_n96()
    dcode = nd.Code(code, windows=(4, 2, 1))
    empty = torch.empty((0, code.n), dtype=torch.float32, device="cuda:0")
    out = nd.decode(dcode, empty, 10)
    torch.cuda.synchronize()
    assert out["hard"].shape == (0, code.n)
    llr, _ = make_frames(code.n, 1, 2.0, 0.5, seed=3)
    g = gpu_decode(dcode, llr, 10, False)
    dcode.close()
    r = oracle.decode_with_sensitivity(code, _groups(code, (4, 2, 1)), llr, 10, False)
    compare(g, r)


def test_largest_code_in_lds_and_one_beyond():
    # n = 8064 QC rate-1/2 code of the serving workload (z = 336, one base
    # row per window, overlap 84): FP32 messages with the default four lanes
    # per CN visit need more lanes per group than a workgroup has, so every
    # group runs in several passes; FP16 messages with their default mapping
    key = W.qc_key(8064, "1/2")
    code = W.CODES[key]()
    win = W.serve_windows(8064, "1/2")
    dcode = nd.Code(code, windows=win)
    info = dcode.info
    assert info["lds_bytes_16"] <= info["lds_limit"] and info["lds_bytes_fp32"] <= info["lds_limit"]
    assert info["lanes_fp32"] == 4 and info["cn_visits"] // info["num_groups"] * 4 > 1024
    groups = _groups(code, win)
    enc = W.encoder_for(key)
    try:
        for eb, seed in ((1.5, 33), (2.5, 34)):
            llr, _ = make_frames(code.n, 64, eb, enc.rate, seed, encoder=enc)
            g = gpu_decode(dcode, llr, 20, True)
            r = oracle.decode_with_sensitivity(code, groups, llr, 20, True)
            print("n=8064 fp32", eb, compare(g, r))
            g16 = gpu_decode(dcode, llr, 20, True, msg="fp16")
            print("n=8064 fp16", eb, compare16(g16, r))
    finally:
        dcode.close()
    print("lds per frame (fp32, 16-bit):", info["lds_bytes_fp32"], info["lds_bytes_16"])
    # n = 60000 (near the largest n the tables address): the posteriors alone
    # exceed the LDS of a workgroup, so the decode takes the HBM tier; it must
    # meet the oracle bar (all-zero codeword, 3 dB)
    big = regular_code(60000, 3, 6, seed=7, girth6=False)
    bcode = nd.Code(big, windows=(8, 40, 1))
    assert bcode.info["lds_bytes_fp32"] > bcode.info["lds_limit"]
    llr, _ = make_frames(big.n, 6, 3.0, 0.5, seed=34)
    g = gpu_decode(bcode, llr, 8, True)
    bcode.close()
    ref = oracle.decode_with_sensitivity(big, _groups(big, (8, 40, 1)), llr, 8, True)
    print("n=60000", compare(g, ref))


def test_repeated_launches_reuse_work_counters():
    """More decode calls than the work-counter ring holds, back to back on one
    stream: every call must see a fresh counter."""
    code = W.code_n96()
    dcode = nd.Code(code, windows=(4, 2, 1))
    llr, _ = make_frames(code.n, 37, 2.0, 0.5, seed=44)
    first = gpu_decode(dcode, llr, 10, True)
    x = torch.from_numpy(llr).to("cuda:0")
    out = None
    for _ in range(1100):
        out = nd.decode(dcode, x, 10, early_stop=True)
    torch.cuda.synchronize()
    dcode.close()
    for k in first:
        assert np.array_equal(out[k].cpu().numpy(), first[k]), k


def test_default_mapping_rule():
    """The built-in CN-lane mapping, chosen at create per message format
    from LDS residency: two lanes for the (3,6) n=2304 code (FP32), four
    (the widest workgroup) for the serving workload's QC n=8064 rate-1/2 code
    with FP32 messages, where every mapping leaves one workgroup per CU; the chosen mapping fits in
    LDS whenever one does, and tuning to 0 restores it."""
    sweep = nd.Code(W.CODES["n2304"](), windows=(8, 16, 1))
    big = nd.Code(W.CODES[W.qc_key(8064, "1/2")](), windows=W.serve_windows(8064, "1/2"))
    try:
        assert sweep.info["lanes_fp32"] == 2
        assert big.info["lanes_fp32"] == 4
        for c in (sweep, big):
            info = c.info
            assert info["lds_bytes_fp32"] <= info["lds_limit"] and info["lds_bytes_16"] <= info["lds_limit"]
            for msg in ("fp32", "fp16", "bf16"):
                base = info["lanes_" + msg]
                assert base in (1, 2, 4)
                c.tune(msg, 1)
                c.tune(msg, 0)
                assert c.info["lanes_" + msg] == base
    finally:
        sweep.close()
        big.close()


def test_tune_arguments():
    """ldpc_code_tune: bad values and unbuilt mappings are errors; 0
    restores the default; each message format keeps its own choice."""
    code = W.CODES["n96"]()
    dcode = nd.Code(code, windows=(4, 2, 1))
    try:
        base = (dcode.info["lanes_fp32"], dcode.info["lanes_fp16"], dcode.info["lanes_bf16"])
        for bad in (3, -1):
            with pytest.raises(nd.LdpcError) as ei:
                dcode.tune("fp32", bad)
            assert ei.value.code == nd.LDPC_EINVAL
        with pytest.raises(nd.LdpcError) as ei:
            nd.ldpc_code_tune(dcode.handle, nd.LDPC_FLAG_MSG_FP16 | nd.LDPC_FLAG_MSG_BF16, 1)
        assert ei.value.code == nd.LDPC_EINVAL
        dcode.tune("bf16", 1)
        assert dcode.info["lanes_bf16"] == 1
        assert (dcode.info["lanes_fp32"], dcode.info["lanes_fp16"]) == base[:2]
        dcode.tune("bf16", 0)
        assert dcode.info["lanes_bf16"] == base[2]
    finally:
        dcode.close()
    # degree 7: one lane runs the exact-degree variant, two lanes pad to 8
    code = regular_code(84, 3, 7, seed=5)
    llr, _ = make_frames(code.n, 64, 2.5, 4 / 7, seed=51)
    for lanes in (1, 2):
        g, r = _run_both(code, (5, 2, 1), llr, 12, True, lanes=lanes)
        print("degree 7, lanes", lanes, compare(g, r))


@pytest.mark.parametrize("lanes", [1, 2, 4])
@pytest.mark.parametrize("msg", ["fp32", "fp16"])
def test_lanes_per_check_node(lanes, msg):
    """Every CN-phase mapping (one lane per CN visit, or two or four lanes
    sharing it), chosen per message format, meets the parity bar on the
    n=2304 workload and on the QC code (FP32 messages: the two-tier bar;
    FP16: the posterior error bound of the 16-bit formats)."""
    for rec, snr in ((W.SWEEP, 2), (W.PRECISION, 0)):
        code = W.CODES[rec["code"]]()
        llr, _ = W.frames(rec, snr, num_frames=96, first_frame=500)
        if msg == "fp16":
            dcode = nd.Code(code, windows=rec["windows"])
            try:
                dcode.tune("fp16", lanes)
                assert dcode.info["lanes_fp16"] == lanes
                g = gpu_decode(dcode, llr, rec["max_iter"], True, "fp16")
            finally:
                dcode.close()
            r = oracle.decode(code, _groups(code, rec["windows"]), llr, rec["max_iter"], True)
            print("lanes", lanes, rec["name"], "fp16", compare16(g, r))
            continue
        g, r = _run_both(code, rec["windows"], llr, rec["max_iter"], True, lanes=lanes)
        print("lanes", lanes, rec["name"], compare(g, r))


def test_step1_random_grouping_meets_bar():
    """The paper's own grouping (Step 1: random groups with overlap ratio
    r = 0.4, G = 12, N_G = 34) on the n=504 stand-in, through explicit groups."""
    from paper_1202_1060_amd.grouping import step1_groups
    code = W.CODES["n504"]()
    groups = step1_groups(code.m, 12, 0.4, np.random.Generator(np.random.Philox(3100)))
    llr, _ = make_frames(code.n, 96, 2.0, 0.5, seed=61)
    dcode = nd.Code(code, groups=groups)
    g = gpu_decode(dcode, llr, 60, True)
    dcode.close()
    ref = oracle.decode_with_sensitivity(code, groups, llr, 60, True)
    print("step1 n504", compare(g, ref))


def test_regrouping_every_iteration_meets_bar():
    """Step 4 returns to Step 1: a new random Step-1 grouping every
    iteration (R = 5 drawn groupings, cycled), against the oracle's schedule;
    a batch gives the same as the single decode; the HBM tier refuses it."""
    from paper_1202_1060_amd.grouping import step1_groups
    code = W.CODES["n504"]()
    rng = np.random.Generator(np.random.Philox(3200))
    sched = []
    for _ in range(5):
        sched += step1_groups(code.m, 12, 0.4, rng)
    llr, _ = make_frames(code.n, 96, 2.0, 0.5, seed=62)
    dcode = nd.Code(code, groups=sched, groups_per_iteration=12)
    assert dcode.info["groups_per_iteration"] == 12 and dcode.info["num_groups"] == 60
    g = gpu_decode(dcode, llr, 23, True)
    ref = oracle.decode_with_sensitivity(code, sched, llr, 23, True, groups_per_iteration=12)
    print("regroup n504", compare(g, ref))
    x = torch.from_numpy(llr).to("cuda:0")
    outs = nd.decode_batched([nd.Problem(dcode, x, 23)], msg="fp32")
    torch.cuda.synchronize()
    for k in ("hard", "post", "iters", "syn_ok"):
        assert np.array_equal(outs[0][k].cpu().numpy(), g[k]), k
    from paper_1202_1060_amd import _native
    o = nd.new_outputs(96, code.n, x.device)
    with pytest.raises(nd.LdpcError) as ei:
        nd.ldpc_decode(dcode.handle, x.data_ptr(), 96, 23, _native.LDPC_FLAG_TIER_HBM, o["hard"].data_ptr(), 0,
                       o["iters"].data_ptr(), 0, torch.cuda.current_stream().cuda_stream)
    assert ei.value.code == nd.LDPC_EUNSUPPORTED
    dcode.close()


def test_degenerate_codes_and_caps():
    """A VN in no check keeps its channel LLR; one iteration; identical
    frames decode identically; a code with a single check of every VN."""
    rows = [[0, 1, 2], [1, 2, 3], [2, 3, 4]]  # VN 5 is in no check
    code = Code.from_rows(rows, 6)
    rng = np.random.default_rng(21)
    llr = rng.normal(1.0, 1.2, size=(1, 6)).astype(np.float32).repeat(40, axis=0)
    dcode = nd.Code(code, windows=(2, 1, 1))
    for it in (1, 5):
        g, r = gpu_decode(dcode, llr, it, False), oracle.decode(code, _groups(code, (2, 1, 1)), llr, it, False)
        assert np.all(g["post"] == g["post"][0])  # identical frames
        np.testing.assert_allclose(g["post"][:, 5], llr[:, 5], rtol=1e-6)
        np.testing.assert_allclose(g["post"], r["post"], rtol=1e-4, atol=1e-3)
        assert np.all(g["iters"] == it)
    dcode.close()
    one = Code.from_rows([list(range(8))], 8)  # one check over all VNs
    llr1 = rng.normal(0.5, 1.0, size=(16, 8)).astype(np.float32)
    dcode = nd.Code(one, windows=(1, 0, 1))
    g = gpu_decode(dcode, llr1, 3, True)
    r = oracle.decode(one, [np.arange(1)], llr1, 3, True)
    np.testing.assert_allclose(g["post"], r["post"], rtol=1e-4, atol=1e-3)
    assert np.array_equal(g["iters"], r["iters"])
    dcode.close()


@pytest.mark.parametrize("lanes", [1, 2])
@pytest.mark.parametrize("which", ["qc_rate_2_3", "regular_5_10"])
def test_degree_ten_variants(which, lanes):
    """Checks of degree 9 and 10 (a rate-2/3 QC code: padded variant D = 10)
    and a (5,10)-regular code (uniform D = 10), both CN-lane mappings."""
    if which == "qc_rate_2_3":
        code = W.CODES["qc1152r2_3"]()
        windows = (9, 12, 1)
        llr, _ = make_frames(code.n, 160, 2.6, 2 / 3, seed=91, encoder=W.encoder_for("qc1152r2_3"))
    else:
        code = regular_code(600, 5, 10, seed=77, girth6=True)
        windows = (6, 8, 1)
        llr, _ = make_frames(code.n, 160, 2.6, 0.5, seed=91)
    assert int(np.diff(code.row_ptr).max()) == 10
    g, r = _run_both(code, windows, llr, 15, True, lanes=lanes)
    print(which, "lanes", lanes, compare(g, r))


@pytest.mark.parametrize("lanes", [1, 2, 4])
@pytest.mark.parametrize("dv,dc,n", [(2, 4, 96), (3, 7, 336), (3, 8, 256), (3, 12, 384), (3, 16, 512),
                                     (4, 24, 480), (4, 32, 512)])
def test_every_uniform_degree_variant(dv, dc, n, lanes):
    """Each padded-degree kernel variant on a regular code whose checks all
    have that degree (the uniform form; degree 7 with two or four lanes runs
    the degree-8 variant with one padding edge per check), with one, two and
    four lanes per CN visit (four: the degree padded to a multiple of 4)."""
    code = regular_code(n, dv, dc, seed=3, girth6=False)
    rate = 1.0 - dv / dc
    llr, _ = make_frames(code.n, 64, 3.0 if dc <= 12 else 4.5, rate, seed=95)
    windows = (4, max(1, code.m // 16), 1)
    g, r = _run_both(code, windows, llr, 12, True, lanes=lanes)
    print((dv, dc, n), "lanes", lanes, compare(g, r))


def _vn_windows(n, G):
    return [np.arange((g * n) // G, ((g + 1) * n) // G, dtype=np.int32) for g in range(G)]


@pytest.mark.parametrize("lanes", [1, 2])
@pytest.mark.parametrize("which", ["sweep_G8", "qc_G12", "n96_singletons", "one_group"])
def test_vertical_schedule_meets_bar(which, lanes):
    """The vertical (VN-group) shuffled schedule, the prior art Sec. I
    contrasts with, on the GPU against the oracle's vertical decoder: the
    sweep code with 8 contiguous VN groups, the rate-1/2 QC code (checks of
    degree 6 and 7) with 12, the n=96 code with one VN per group, and one
    group of every VN (flooding)."""
    if which == "sweep_G8":
        rec = W.SWEEP
        code = W.CODES[rec["code"]]()
        llr, _ = W.frames(rec, 2, num_frames=96, first_frame=300)
        vg, it = _vn_windows(code.n, 8), 20
    elif which == "qc_G12":
        rec = W.PRECISION
        code = W.CODES[rec["code"]]()
        llr, _ = W.frames(rec, 0, num_frames=96, first_frame=40)
        vg, it = _vn_windows(code.n, 12), 15
    elif which == "n96_singletons":
        code = W.code_n96()
        llr, _ = make_frames(code.n, 64, 2.0, 0.5, seed=97)
        vg, it = [[v] for v in np.random.default_rng(5).permutation(code.n)], 6
    else:
        code = W.code_n96()
        llr, _ = make_frames(code.n, 64, 2.0, 0.5, seed=98)
        vg, it = [np.arange(code.n)], 10
    dcode = nd.Code(code, vn_groups=vg)
    try:
        dcode.tune("fp32", lanes)
        g = gpu_decode(dcode, llr, it, True)
    finally:
        dcode.close()
    r = oracle.decode_vertical_with_sensitivity(code, vg, llr, it, True)
    print(which, "lanes", lanes, compare(g, r))


def test_vertical_schedule_fp16_and_refusals():
    """FP16 messages meet the 16-bit bar; the HBM tier, BF16
    messages, four lanes and batches refuse VN groups."""
    from paper_1202_1060_amd import _native
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    llr, _ = W.frames(rec, 3, num_frames=64, first_frame=800)
    vg = _vn_windows(code.n, 8)
    dcode = nd.Code(code, vn_groups=vg)
    try:
        g = gpu_decode(dcode, llr, 20, True, "fp16")
        r = oracle.decode_vertical(code, vg, llr, 20, True)
        print("vertical fp16", compare16(g, r))
        x = torch.from_numpy(llr).to("cuda:0")
        with pytest.raises(nd.LdpcError) as ei:
            nd.decode(dcode, x, 20, msg="bf16")
        assert ei.value.code == nd.LDPC_EUNSUPPORTED
        with pytest.raises(nd.LdpcError) as ei:
            dcode.tune("fp32", 4)
            nd.decode(dcode, x, 20)
        assert ei.value.code == nd.LDPC_EUNSUPPORTED
        dcode.tune("fp32", 0)
        out = nd.new_outputs(x.shape[0], code.n, x.device)
        flags = nd.LDPC_FLAG_EARLY_STOP | _native.LDPC_FLAG_TIER_HBM
        with pytest.raises(nd.LdpcError) as ei:
            nd.ldpc_decode(dcode.handle, x.data_ptr(), x.shape[0], 20, flags, out["hard"].data_ptr(),
                           out["post"].data_ptr(), out["iters"].data_ptr(), out["syn_ok"].data_ptr(),
                           torch.cuda.current_stream().cuda_stream)
        assert ei.value.code == nd.LDPC_EUNSUPPORTED
        with pytest.raises(nd.LdpcError) as ei:
            nd.Batch([nd.Problem(dcode, x, 20)], msg="fp32")
        assert ei.value.code == nd.LDPC_EUNSUPPORTED
    finally:
        dcode.close()
