"""Batched decoding (ldpc_batch_* / ldpc_decode_batched) on the GPU.

Every problem of a batch must give exactly what ldpc_decode gives on it
alone with the same message format and CN-lane mapping (the kernels run the
same arithmetic per frame), whatever the launch options; FP32 batches meet
the oracle bar; graph replays and repeated launches give the eager result.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - needs a GPU
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1202_1060_amd as nd  # noqa: E402
from ldpcgen import workloads as W  # noqa: E402

from parity import gpu_decode, compare, syndrome_zero  # noqa: E402

DEV = torch.device("cuda:0")


def _mixed(count, max_frames, seed_shift=0):
    """A mix of the batched workload's problems with small frame counts
    (every length and rate, 6..16 windows), plus a problem with no frames."""
    probs = W.batch_problems(count=count + seed_shift)[seed_shift:]
    # make sure all four lengths and all three rates appear
    for i, (n, r) in enumerate(zip(W.BATCH_N, W.BATCH_RATES + ("1/2",))):
        probs[i] = dict(probs[i], code=W.qc_key(n, r), n=n, rate=r, windows=(probs[i]["windows"][0], n // 96, 1))
    for i, p in enumerate(probs):
        p["frames"] = 1 + (p["frames"] * 7 + i) % max_frames
        p["max_iter"] = (20, 15, 9, 20)[i % 4]
    probs[3] = dict(probs[3], frames=0)
    return probs


class _Set:
    def __init__(self, specs):
        self.specs = specs
        self.codes, self.llr, self.cw = [], [], []
        for p in specs:
            self.codes.append(nd.Code(W.CODES[p["code"]](), windows=p["windows"]))
            llr, cw = W.problem_frames(p)
            self.llr.append(llr)
            self.cw.append(cw)
        self.dllr = [torch.from_numpy(x).to(DEV) for x in self.llr]

    def problems(self):
        return [nd.Problem(c, x, p["max_iter"]) for c, x, p in zip(self.codes, self.dllr, self.specs)]

    def close(self):
        for c in self.codes:
            c.close()


@pytest.fixture(scope="module")
def mixed():
    s = _Set(_mixed(14, 40))
    yield s
    s.close()


def _host(out):
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def _single(s, i, msg, early_stop=True):
    p = s.specs[i]
    return gpu_decode(s.codes[i], s.llr[i], p["max_iter"], early_stop, msg)


@pytest.mark.parametrize("msg", ["fp16", "fp32", "bf16"])
@pytest.mark.parametrize("opts", [(0, 1, 0, 4), (0, 0, 0, 1), (1, 1, 128, 2), (2, 0, 256, 8), (4, 1, 512, 4)])
def test_batch_equals_single_decodes(mixed, msg, opts):
    o = nd.BatchOptions.from_tuple(opts)
    lanes = o.lanes_per_cn
    if lanes:
        for c in mixed.codes:
            c.tune(msg, lanes)
    try:
        probs = mixed.problems()
        b = nd.Batch(probs, msg=msg, early_stop=True, options=o)
        print(msg, o, b.info)
        b.launch()
        torch.cuda.synchronize()
        b.close()
        for i, p in enumerate(probs):
            got = _host(p.out)
            want = _single(mixed, i, msg)
            for k in want:
                assert np.array_equal(got[k], want[k]), (i, k)
            code = W.CODES[mixed.specs[i]["code"]]()
            if len(got["hard"]):
                assert np.array_equal(got["syn_ok"].astype(bool), syndrome_zero(code, got["hard"])), i
    finally:
        if lanes:
            for c in mixed.codes:
                c.tune(msg, 0)


def test_batch_meets_oracle_bar_fp32(mixed):
    probs = mixed.problems()
    outs = nd.decode_batched(probs, msg="fp32", early_stop=True)
    torch.cuda.synchronize()
    for i, p in enumerate(mixed.specs):
        if p["frames"] == 0:
            continue
        code = W.CODES[p["code"]]()
        groups = oracle.windows(code.m, p["windows"][0], p["windows"][1], True)
        ref = oracle.decode_with_sensitivity(code, groups, mixed.llr[i], p["max_iter"], True)
        print(i, p["code"], p["windows"], compare(_host(outs[i]), ref))


def test_batch_graph_replays(mixed):
    """The batch launch captured in a graph: every replay (with eager work
    and synchronisation between replays) equals the eager launch."""
    probs = mixed.problems()
    b = nd.Batch(probs, msg="fp16", early_stop=True)
    b.launch()
    torch.cuda.synchronize()
    eager = [_host(p.out) for p in probs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            b.launch(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for p in probs:
            for v in p.out.values():
                if v is not None:
                    v.fill_(7)
        junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i, p in enumerate(probs):
            got = _host(p.out)
            for k in eager[i]:
                assert np.array_equal(got[k], eager[i][k]), (rep, i, k)
    del g
    b.close()


def test_batch_repeated_launches(mixed):
    probs = mixed.problems()
    b = nd.Batch(probs, msg="fp16", early_stop=False)
    b.launch()
    torch.cuda.synchronize()
    first = [_host(p.out) for p in probs]
    for _ in range(5):
        b.launch()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        got = _host(p.out)
        for k in first[i]:
            assert np.array_equal(got[k], first[i][k]), (i, k)
        if mixed.specs[i]["frames"]:
            assert np.all(got["iters"] == mixed.specs[i]["max_iter"])
    b.close()


def test_batch_rejects_codes_on_two_devices_and_bad_options(mixed):
    probs = mixed.problems()
    with pytest.raises(nd.LdpcError) as ei:
        nd.Batch(probs, options=nd.BatchOptions(max_threads=100))
    assert ei.value.code == nd.LDPC_EINVAL
    bad = nd.Problem(mixed.codes[0], mixed.dllr[0], 0)
    with pytest.raises(nd.LdpcError) as ei:
        nd.Batch([bad])
    assert ei.value.code == nd.LDPC_EINVAL


def test_single_decode_many_frames_per_workgroup_fixed_iterations():
    """Fixed iterations (20, even) with several frames per persistent
    workgroup, failing and decodable frames interleaved: syn_ok must be the
    syndrome of the returned decisions for every frame."""
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    lo, _ = W.frames(rec, 0, num_frames=1536)
    hi, _ = W.frames(rec, 6, num_frames=1536)
    llr = np.empty((3072, code.n), dtype=np.float32)
    llr[0::2], llr[1::2] = lo, hi
    dcode = nd.Code(code, windows=rec["windows"])
    for es in (False, True):
        g = gpu_decode(dcode, llr, rec["max_iter"], es)
        ok = syndrome_zero(code, g["hard"])
        assert np.array_equal(g["syn_ok"].astype(bool), ok), es
        assert 0 < ok.sum() < len(ok)
        print("early stop", es, "decoded", ok.mean())
    dcode.close()


def test_autotuner_picks_and_caches(mixed, tmp_path):
    from paper_1202_1060_amd import autotune
    probs = mixed.problems()
    cache = str(tmp_path / "tune.json")
    cands = [nd.BatchOptions(0, 1, 0, 4), nd.BatchOptions(1, 0, 256, 1), nd.BatchOptions(2, 1, 0, 2)]
    try:
        best = autotune.tune_batch(probs, msg="fp16", cache=cache, candidates=cands, reps=2)
        assert best.as_tuple() in [c.as_tuple() for c in cands]
        tuned = [c.info["lanes_fp16"] for c in mixed.codes]
        assert set(tuned) <= {1, 2, 4}
        for c in mixed.codes:
            c.tune("fp16", 0)
        # the cached answer restores the per-code lanes too
        again = autotune.tune_batch(probs, msg="fp16", cache=cache, candidates=[])
        assert again.as_tuple() == best.as_tuple()
        assert [c.info["lanes_fp16"] for c in mixed.codes] == tuned
        lanes = autotune.tune_code(mixed.codes[1], mixed.dllr[1], 20, msg="fp32", cache=cache, reps=2)
        assert lanes in (1, 2, 4) and mixed.codes[1].info["lanes_fp32"] == lanes
    finally:
        for c in mixed.codes:
            c.tune("fp32", 0)
            c.tune("fp16", 0)


def test_async_batched_calls_in_flight(mixed):
    """40 asynchronous ldpc_decode_batched calls (more than the 16 staging
    slots) on two streams without host synchronisation, each on a different
    subset of the problems with its own outputs: every output equals the
    single decode of its problem."""
    rng = np.random.default_rng(3)
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    streams[1].wait_stream(streams[0])
    calls = []
    for c in range(40):
        idx = sorted(rng.choice(len(mixed.specs), size=int(rng.integers(1, 6)), replace=False).tolist())
        probs = [nd.Problem(mixed.codes[i], mixed.dllr[i], mixed.specs[i]["max_iter"]) for i in idx]
        nd.decode_batched(probs, msg="fp16", stream=streams[c % 2])
        calls.append((idx, probs))
    torch.cuda.synchronize()
    want = {i: _single(mixed, i, "fp16") for i in range(len(mixed.specs))}
    for idx, probs in calls:
        for i, p in zip(idx, probs):
            got = _host(p.out)
            for k in want[i]:
                assert np.array_equal(got[k], want[i][k]), (idx, i, k)


def test_packed_hard_decisions(mixed):
    """LDPC_FLAG_OUT_PACKED: byte q bit k = d_{8q+k}, bits past n zero; the
    same decisions as the byte-per-bit layout, single and batched."""
    for i in (0, 1, 6):
        p = mixed.specs[i]
        ref = _single(mixed, i, "fp16")
        got = nd.decode(mixed.codes[i], mixed.dllr[i], p["max_iter"], msg="fp16", packed=True)
        torch.cuda.synchronize()
        hb = got["hard"].cpu().numpy()
        n = mixed.codes[i].n
        assert hb.shape == (p["frames"], (n + 7) // 8)
        assert np.array_equal(np.unpackbits(hb, axis=1, bitorder="little")[:, :n], ref["hard"])
        assert not np.any(np.unpackbits(hb, axis=1, bitorder="little")[:, n:])
        for k in ("post", "iters", "syn_ok"):
            assert np.array_equal(got[k].cpu().numpy(), ref[k])
    probs = [nd.Problem(c, x, p["max_iter"], packed=True) for c, x, p in zip(mixed.codes, mixed.dllr, mixed.specs)]
    nd.decode_batched(probs, msg="fp16")
    torch.cuda.synchronize()
    for i, pr in enumerate(probs):
        n = mixed.codes[i].n
        ref = _single(mixed, i, "fp16")
        hb = pr.out["hard"].cpu().numpy()
        assert np.array_equal(np.unpackbits(hb, axis=1, bitorder="little")[:, :n], ref["hard"]), i
