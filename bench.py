"""Throughput of NDGSBP decoding on one MI355X.

Workload (one step): the (3,6)-regular n=2304 code (m=1152, 4-cycle-free,
seeded), 8 CN windows of 160 CNs with a 16-CN overlap (wraparound), 16384
frames of random information bits at each Eb/N0 in 1.0, 1.25, ..., 2.5 dB
(114688 frames), BPSK/AWGN, at most 20 iterations with the syndrome stop of
Step 4. All LLRs are resident in HBM before timing starts; one step is one
decode call over all frames (hard decisions, posteriors, iteration counts
and syndrome flags written back to HBM).

Prints one JSON line. The decoded info rate counts K = 1152 information bits
per frame. The roofline object is for the decode kernel, bound by VALU issue
(34 full-rate slots per edge update against the chip's FP32 vector peak,
derived below; beside it the fraction of the bound that the measured issue
rates of plain FP32 code give). Further legs in the same line: fixed
iterations, FP16 messages, the same frames under the baseline schedules
(flooding BP, disjoint GSBP, vertical GSBP), the 256-problem mixed batch
(FP16 and FP32 messages) against one FP32 launch per problem, the HBM tier,
and request serving with continuous batching (p50/p99 latency, LLRs resident
in device memory or staged from pinned host memory) against one FP32 launch
per request.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded info Gbit/s at matched FER (served/batched vs plain); p50/p99 latency"

# VALU work per edge update that the method itself needs, in full-rate FP32
# issue slots: two phi evaluations of one exp, one log and one reciprocal
# each (6 transcendentals, a quarter of the FP32 rate, 4 slots each) and
# about ten full-rate ops (extrinsic, clamp, exclusive sums, sign, add-back):
# 6 * 4 + 10 = 34.
SLOTS_PER_EDGE_UPDATE = 34
TRANSCENDENTALS_PER_EDGE_UPDATE = 6
FULL_RATE_PER_EDGE_UPDATE = 10
# Peak from the chip's figures: FP32 vector 157.3 TFLOP/s = 256 CUs x 2.4 GHz
# x 128 FMA lane-slots per CU-cycle = 78.6 T slots/s (an FMA is one slot)
PEAK_SLOTS_PER_S = 256 * 128 * 2.4e9
# Issue rates measured on MI355X by the probes of --calibrate-valu (the
# fastest of repeated runs; FMA with 16 independent chains per lane,
# exp2 + log2 with 8): a second bound from what plain FP32 code attains,
# transcendentals and full-rate ops sharing the issue slots (the mixed
# probe takes 1.02 x the sum of its parts)
MEASURED_FMA_PER_S = 55.90e12
MEASURED_TRANS_PER_S = 17.82e12
EDGE_UPDATES_PER_S_MEASURED_BOUND = 1.0 / (TRANSCENDENTALS_PER_EDGE_UPDATE / MEASURED_TRANS_PER_S
                                           + FULL_RATE_PER_EDGE_UPDATE / MEASURED_FMA_PER_S)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_key(paths):
    """sha1 of the kernel sources with comments and white space removed: a
    comment edit leaves the key (and the device code) as it was, any change
    to the code gives a new key."""
    import hashlib
    import re
    h = hashlib.sha1()
    for p in paths:
        text = open(os.path.join(ROOT, p)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(msg):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    record, if it was taken on the kernel code as it is now (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_n2304_sweep.json")
    if msg != "fp32" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if kernel_sources_key(rec["kernel_sources"]) != rec["kernel_sources_key"]:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def make_inputs(rec, frames_per_snr):
    from ldpcgen import workloads as W
    llrs, cws = [], []
    for i in range(len(rec["ebn0"])):
        llr, cw = W.frames(rec, i, num_frames=frames_per_snr)
        llrs.append(llr)
        cws.append(cw)
    return np.concatenate(llrs), np.concatenate(cws)


def physical_cores():
    """Physical cores of the host (distinct core/socket pairs of lscpu), or None."""
    import subprocess
    try:
        out = subprocess.run(["lscpu", "-p=core,socket"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    pairs = {line.strip() for line in out.splitlines() if line and not line.startswith("#")}
    return len(pairs) or None


def cpu_baseline(code, groups, llr, rec, frames_per_snr, seconds, k_info, gpu_hard=None):
    """The FP64 oracle on the host cores over a bounded sample of the same
    workload: the first F frames of every Eb/N0 point, F sized by a pilot run
    of 16 frames per point so that the timed run takes about ``seconds``;
    then a one-thread run over a quarter of that sample, and the one-ulp
    sensitivity control (the same frames with every LLR moved by one float32
    ulp) whose decision changes are reported per Eb/N0 beside the GPU's
    decision mismatches on the same frames."""
    import oracle
    points = len(rec["ebn0"])

    def sample(per_snr):
        return np.concatenate([np.arange(per_snr) + i * frames_per_snr for i in range(points)])

    pilot = min(16, frames_per_snr)
    t0 = time.perf_counter()
    oracle.decode(code, groups, llr[sample(pilot)], rec["max_iter"], rec["early_stop"], nthreads=0)
    per_snr = int(min(frames_per_snr, max(pilot, pilot * seconds / max(time.perf_counter() - t0, 1e-6))))
    idx = sample(per_snr)
    t0 = time.perf_counter()
    out = oracle.decode(code, groups, llr[idx], rec["max_iter"], rec["early_stop"], nthreads=0)
    dt = time.perf_counter() - t0
    # one thread, a quarter of the sample
    per1 = max(1, per_snr // 4)
    idx1 = sample(per1)
    t0 = time.perf_counter()
    one = oracle.decode(code, groups, llr[idx1], rec["max_iter"], rec["early_stop"], nthreads=1)
    dt1 = time.perf_counter() - t0
    # sensitivity control on the all-thread sample
    ctl = oracle.decode(code, groups, oracle.perturb_one_ulp(llr[idx]), rec["max_iter"], rec["early_stop"],
                        nthreads=0)
    rows = []
    for i, eb in enumerate(rec["ebn0"]):
        sl = slice(i * per_snr, (i + 1) * per_snr)
        ref_h = out["hard"][sl]
        row = {"ebn0": eb, "frames": per_snr, "oracle_decoded": int(out["syn_ok"][sl].sum()),
               "control_decision_changes": int(np.any(ctl["hard"][sl] != ref_h, axis=1).sum())}
        if gpu_hard is not None:
            row["gpu_decision_mismatches"] = int(np.any(gpu_hard[idx[sl]] != ref_h, axis=1).sum())
        rows.append(row)
    return dict(value=len(idx) * k_info / dt / 1e9, unit="Gbit/s", cores=int(out["threads"]),
                kind="oracle",
                sample=f"first {per_snr} frames of each of the {points} Eb/N0 "
                       f"points ({len(idx)} frames), FP64, {dt:.1f} s",
                seconds=dt, logical_cpus=os.cpu_count(), physical_cores=physical_cores(),
                one_thread={"value": len(idx1) * k_info / dt1 / 1e9, "unit": "Gbit/s", "cores": int(one["threads"]),
                            "sample": f"first {per1} frames of each Eb/N0 point ({len(idx1)} frames), {dt1:.1f} s",
                            "frames_per_s": len(idx1) / dt1},
                frames_per_s=len(idx) / dt, sensitivity_control=rows)


def clopper_pearson(k, n, alpha=0.05):
    from scipy.stats import beta
    lo = 0.0 if k == 0 else float(beta.ppf(alpha / 2, k, n - k + 1))
    hi = 1.0 if k == n else float(beta.ppf(1 - alpha / 2, k + 1, n - k))
    return lo, hi


def bench_batched(args, torch, nd, W, dev, log):
    """Mixed batch of 256 QC problems: one FP16 batch plan (autotuned launch
    options) against a plain FP32 ldpc_decode per problem, same frames."""
    from paper_1202_1060_amd import autotune
    rec = W.BATCH
    specs = W.batch_problems(rec)
    t0 = time.perf_counter()
    codes, llrs, cws, ks = [], [], [], []
    cache = {}
    for p in specs:
        llr, cw = W.problem_frames(p)
        if p["code"] not in cache:
            cache[p["code"]] = W.CODES[p["code"]]()
        codes.append(nd.Code(cache[p["code"]], windows=p["windows"]))
        llrs.append(torch.from_numpy(llr).to(dev))
        cws.append(cw)
        ks.append(W.encoder_for(p["code"]).k)
    frames = np.array([p["frames"] for p in specs])
    bits = float(np.dot(frames, ks))
    log(f"batched inputs: {len(specs)} problems, {frames.sum()} frames in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream(dev)

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        evs = []
        t0 = time.perf_counter()
        for _ in range(steps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            evs.append((a, b))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        return wall, float(np.median([a.elapsed_time(b) for a, b in evs]))

    e_iter = [c.info["edge_updates"] for c in codes]

    def fer(outs):
        err = sum(int(np.any(o["hard"].cpu().numpy() != cw, axis=1).sum()) for o, cw in zip(outs, cws))
        its = [int(o["iters"].sum()) for o in outs]
        it = float(sum(its)) / frames.sum()
        lo, hi = clopper_pearson(err, int(frames.sum()))
        return dict(fer=err / frames.sum(), frame_errors=err, ci95=[lo, hi], mean_iters=it,
                    edge_updates=float(np.dot(its, e_iter)))

    probs = [nd.Problem(c, x, p["max_iter"], want_post=False) for c, x, p in zip(codes, llrs, specs)]
    t0 = time.perf_counter()
    opts = autotune.tune_batch(probs, msg=rec["msg"], early_stop=rec["early_stop"],
                               cache=args.tune_cache)
    lane_use = {}  # CN-lane mapping each problem runs with in the batch
    for p in probs:
        h = opts.lanes_per_cn or p.code.info["lanes_" + rec["msg"]]
        lane_use[h] = lane_use.get(h, 0) + 1
    log(f"batched options {opts}, problems per CN-lane mapping {dict(sorted(lane_use.items()))} "
        f"({time.perf_counter() - t0:.1f} s)")
    batch = nd.Batch(probs, msg=rec["msg"], early_stop=rec["early_stop"], options=opts)
    bwall, bms = timed(lambda: batch.launch(stream), args.batch_steps)
    bstats = fer([p.out for p in probs])
    info = batch.info
    # the same batch captured once in a graph and replayed
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            batch.launch(side)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    gwall, gms = timed(graph.replay, args.batch_steps)
    gstats = fer([p.out for p in probs])
    del graph
    batch.close()

    # the same batch with FP32 messages (precision separated from batching)
    probs32 = [nd.Problem(c, x, p["max_iter"], want_post=False) for c, x, p in zip(codes, llrs, specs)]
    opts32 = autotune.tune_batch(probs32, msg="fp32", early_stop=rec["early_stop"], cache=args.tune_cache)
    batch32 = nd.Batch(probs32, msg="fp32", early_stop=rec["early_stop"], options=opts32)
    b32wall, b32ms = timed(lambda: batch32.launch(stream), args.batch_steps)
    b32stats = fer([p.out for p in probs32])
    b32info = batch32.info
    batch32.close()
    log(f"batched fp32 options {opts32}: {bits / (b32ms * 1e-3) / 1e9:.2f} Gbit/s")

    plain_out = [nd.new_outputs(p["frames"], c.n, dev, want_post=False) for p, c in zip(specs, codes)]

    def plain():
        for c, x, p, o in zip(codes, llrs, specs, plain_out):
            nd.decode(c, x, p["max_iter"], early_stop=rec["early_stop"], msg="fp32", out=o, stream=stream)

    pwall, pms = timed(plain, max(1, args.batch_steps // 2))
    pstats = fer(plain_out)
    for c in codes:
        c.close()
    return {
        "workload": "256 QC problems, n in {576,1152,2304,4608}, R in {1/2,2/3,3/4}, z=n/24, "
                    "64-1024 frames (log-uniform), Eb/N0 U[1,3] dB, 6-16 windows with overlap z/4, "
                    "I_max 20, syndrome stop",
        "frames": int(frames.sum()), "info_bits": bits,
        "batched_fp16": {"gbit_s": bits / (bms * 1e-3) / 1e9, "ms": bms, "wall_ms": bwall * 1e3,
                         "edge_updates_per_s": bstats["edge_updates"] / (bms * 1e-3),
                         "roofline_frac": bstats["edge_updates"] * SLOTS_PER_EDGE_UPDATE / (bms * 1e-3)
                         / PEAK_SLOTS_PER_S,
                         "launches": info["num_launches"], "streams": info["num_streams"],
                         "options": list(opts.as_tuple()),
                         "problems_per_lane_mapping": {str(k): v for k, v in sorted(lane_use.items())},
                         **bstats},
        "batched_fp16_graph_replay": {"gbit_s": bits / (gms * 1e-3) / 1e9, "ms": gms, "wall_ms": gwall * 1e3,
                                      "frame_errors": gstats["frame_errors"]},
        "batched_fp32": {"gbit_s": bits / (b32ms * 1e-3) / 1e9, "ms": b32ms, "wall_ms": b32wall * 1e3,
                         "edge_updates_per_s": b32stats["edge_updates"] / (b32ms * 1e-3),
                         "roofline_frac": b32stats["edge_updates"] * SLOTS_PER_EDGE_UPDATE / (b32ms * 1e-3)
                         / PEAK_SLOTS_PER_S,
                         "launches": b32info["num_launches"], "options": list(opts32.as_tuple()), **b32stats},
        "plain_fp32_per_problem": {"gbit_s": bits / (pms * 1e-3) / 1e9, "ms": pms, "wall_ms": pwall * 1e3,
                                   "edge_updates_per_s": pstats["edge_updates"] / (pms * 1e-3),
                                   "launches": len(specs), **pstats},
        "speedup": pms / bms,
    }


def bench_hbm(args, torch, nd, W, dev, log, sweep_llr, sweep_k):
    """HBM tier: the sweep frames forced into the HBM tier, and a code beyond
    LDS (QC rate 1/2, n=16896, 12 windows, overlap 176; all-zero codeword at
    2.0 dB). Algorithmic HBM bytes per edge update: posterior read + write
    (8 B) + message read + write (2 x message size)."""
    from paper_1202_1060_amd import _native
    from ldpcgen.codes import qc_code, base_mask
    stream = torch.cuda.current_stream(dev)

    def run(dcode, x, max_iter, msg, steps, force):
        F = x.shape[0]
        out = nd.new_outputs(F, dcode.n, dev, want_post=False)
        flags = (nd.msg_flag(msg) | nd.LDPC_FLAG_EARLY_STOP | (_native.LDPC_FLAG_TIER_HBM if force else 0))

        def once():
            nd.ldpc_decode(dcode.handle, x.data_ptr(), F, max_iter, flags, out["hard"].data_ptr(), 0,
                           out["iters"].data_ptr(), out["syn_ok"].data_ptr(), stream.cuda_stream)
        once()
        torch.cuda.synchronize()
        evs = []
        for _ in range(steps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            once()
            b.record(stream)
            evs.append((a, b))
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
        iters = out["iters"].cpu().numpy()
        eu = float(iters.astype(np.int64).sum()) * dcode.info["edge_updates"]
        mb = 4 if msg == "fp32" else 2
        gbs = eu * (8 + 2 * mb) / (ms * 1e-3) / 1e9
        return dict(ms=ms, edge_updates_per_s=eu / (ms * 1e-3), mean_iters=float(iters.mean()),
                    algorithmic_gb_s=gbs, hbm_frac=gbs / 8000.0), iters

    rec = W.SWEEP
    out = {"bytes_per_edge_update": "8 + 2 x message bytes"}
    code = W.CODES[rec["code"]]()
    dcode = nd.Code(code, windows=rec["windows"])
    x = torch.from_numpy(sweep_llr).to(dev)
    for msg in ("fp32", "fp16"):
        r, iters = run(dcode, x, rec["max_iter"], msg, args.hbm_steps, True)
        r["gbit_s"] = x.shape[0] * sweep_k / (r["ms"] * 1e-3) / 1e9
        out[f"sweep_forced_{msg}"] = r
        log(f"hbm tier, sweep {msg}: {r['gbit_s']:.2f} Gbit/s, {r['algorithmic_gb_s']:.0f} GB/s")
    dcode.close()
    del x
    big = qc_code(base_mask("1/2", 1030), 704, 1030)
    bcode = nd.Code(big, windows=(12, 176, 1))
    # all-zero codeword over BPSK/AWGN at 2.0 dB (rate 1/2), drawn on the
    # device: 131072 frames are 8.9 GB of LLRs
    sigma = float(np.sqrt(1.0 / (2 * 0.5 * 10 ** (2.0 / 10))))
    gen = torch.Generator(device=dev)
    gen.manual_seed(1031)
    x = (2.0 / sigma ** 2) * (1.0 + sigma * torch.randn(args.hbm_big_frames, big.n, device=dev, generator=gen))
    for msg in ("fp32", "fp16"):
        r, _ = run(bcode, x, 20, msg, args.hbm_steps, False)
        r["gbit_s"] = x.shape[0] * (big.n - big.m) / (r["ms"] * 1e-3) / 1e9
        out[f"n16896_{msg}"] = r
        log(f"hbm tier, n=16896 {msg}: {r['gbit_s']:.2f} Gbit/s, {r['algorithmic_gb_s']:.0f} GB/s")
    out["n16896"] = {"frames": int(x.shape[0]), "lds_bytes_fp32": bcode.info["lds_bytes_fp32"],
                     "lds_limit": bcode.info["lds_limit"], "info_bits_per_frame": big.n - big.m,
                     "note": "all-zero codeword, 2.0 dB (LLRs drawn on the device), 12 windows overlap 176, "
                             "I_max 20, syndrome stop; info bits at the design rate (n - m)"}
    bcode.close()
    return out


def serving_frames(torch, W, dev, r, pool, codes):
    """LLRs of every request of the serving stream at its own Eb/N0 (drawn
    continuously from U[1.5, 3.5] dB): request i takes pool rows
    off_i .. off_i + F_i - 1 of its code's channel pool (codewords and unit
    noise, ldpcgen.workloads.serve_symbols) at sigma_i, L = (2/sigma^2)
    (x + sigma w). Built on the device into one float32 buffer holding the
    requests back to back in arrival order. Returns (buffer, element offsets,
    pool row offsets, codeword pools)."""
    from ldpcgen.channel import ebn0_to_sigma
    N = len(r["frames"])
    nvec = np.array([c.n for c in codes], dtype=np.int64)
    F = r["frames"]
    off = np.minimum((r["u"] * (pool - F + 1)).astype(np.int64), pool - F)
    elems = F * nvec[r["code"]]
    host_off = np.concatenate([[0], np.cumsum(elems)])
    buf = torch.empty(int(host_off[-1]), dtype=torch.float32, device=dev)
    cws = []
    for ci, (n, rate) in enumerate(W.SERVE_CODES):
        cw, w = W.serve_symbols(ci, pool)
        cws.append(cw)
        x = torch.from_numpy(1.0 - 2.0 * cw.astype(np.float32)).to(dev)
        wn = torch.from_numpy(w).to(dev)
        idx = np.nonzero(r["code"] == ci)[0]
        if len(idx) == 0:
            continue
        enc_rate = W.encoder_for(W.qc_key(n, rate)).rate
        sig = np.array([ebn0_to_sigma(float(e), enc_rate) for e in r["ebn0"][idx]], dtype=np.float64)
        # one entry per frame: pool row, scales and destination offset
        fr = F[idx]
        rows = np.concatenate([np.arange(o, o + f) for o, f in zip(off[idx], fr)])
        a = np.repeat(2.0 / sig ** 2, fr).astype(np.float32)
        bsc = np.repeat(2.0 / sig, fr).astype(np.float32)
        dst = np.concatenate([h + n * np.arange(f) for h, f in zip(host_off[idx], fr)])
        ar = torch.arange(n, device=dev)
        for c0 in range(0, len(rows), 4096):
            sl = slice(c0, c0 + 4096)
            rt = torch.from_numpy(rows[sl]).to(dev)
            vals = torch.from_numpy(a[sl]).to(dev)[:, None] * x[rt] + torch.from_numpy(bsc[sl]).to(dev)[:, None] * wn[rt]
            d = (torch.from_numpy(dst[sl]).to(dev)[:, None] + ar[None, :]).reshape(-1)
            buf.index_copy_(0, d, vals.reshape(-1))
        del x, wn
    torch.cuda.synchronize()
    return buf, host_off, off, cws


def bench_serving(args, torch, nd, W, dev, log):
    """Serving over the three resident QC codes, requests at continuous
    Eb/N0. Two legs on the same request stream: LLRs already in device
    memory, and LLRs arriving in pinned host memory as FP16 (staged to the
    device by one copy per launch, inside each request's latency). Per leg:
    saturated throughput of the continuous-batching server and of the
    per-request FP32 policy; Poisson arrivals at 0.5x and 0.8x of each
    policy's own saturated rate (p50/p99), and the per-request policy at the
    batched server's offered load; frame error rates of both policies."""
    from paper_1202_1060_amd.serve import Server, Requests
    P = args.serve_pool
    N = args.serve_requests
    t0 = time.perf_counter()
    codes, ks = [], []
    for ci, (n, rate) in enumerate(W.SERVE_CODES):
        key = W.qc_key(n, rate)
        ks.append(W.encoder_for(key).k)
        codes.append(nd.Code(W.CODES[key](), windows=W.serve_windows(n, rate)))
    r = W.serve_requests(count=N)
    buf, host_off, off, cws = serving_frames(torch, W, dev, r, P, codes)
    host = torch.empty(buf.numel(), dtype=torch.float16, pin_memory=True)
    for c0 in range(0, buf.numel(), 1 << 28):
        host[c0:c0 + (1 << 28)].copy_(buf[c0:c0 + (1 << 28)].half())
    torch.cuda.synchronize()
    log(f"serving frames: {int(r['frames'].sum())} frames of {N} requests, {buf.numel() * 4 / 1e9:.2f} GB FP32 "
        f"on the device, {host.numel() * 2 / 1e9:.2f} GB FP16 pinned on the host, in {time.perf_counter() - t0:.1f} s")
    kvec = np.array(ks, dtype=np.int64)
    bits = r["frames"] * kvec[r["code"]]
    max_iter = np.full(N, W.SERVE["max_iter"], dtype=np.int32)
    addr = np.uint64(buf.data_ptr()) + (4 * host_off[:-1]).astype(np.uint64)

    def stream_at(rate, count, staged):
        arr = np.zeros(count) if rate is None else r["arrival"][:count] / rate
        if staged:
            return Requests(arr, r["code"][:count], r["frames"][:count], None, max_iter[:count],
                            host_llr=host, host_off=host_off[:count + 1])
        return Requests(arr, r["code"][:count], r["frames"][:count], addr[:count], max_iter[:count])

    def fer(res, count):
        err = 0
        for i in range(count):
            c, o, F = int(r["code"][i]), int(off[i]), int(r["frames"][i])
            err += int(np.any(res[i]["hard"] != cws[c][o:o + F], axis=1).sum())
        tot = int(r["frames"][:count].sum())
        lo, hi = clopper_pearson(err, tot)
        return dict(fer=err / tot, frame_errors=err, frames=tot, ci95=[lo, hi])

    def summary(o, count):
        return {"requests": count, "p50_ms": o["p50_ms"], "p99_ms": o["p99_ms"],
                "gbit_s": float(bits[:count].sum()) / o["makespan"] / 1e9, "launches": o["launches"]}

    out = {"workload": "3 resident QC codes (n=648 R=5/6, n=1944 R=1/2, n=8064 R=1/2, z=n/24, one base row "
                       "per window, overlap floor(z/4)); Poisson arrivals; requests of 1-512 frames "
                       "(geometric, mean 32), Eb/N0 U[1.5,3.5] dB drawn per request, I_max 20, syndrome stop",
           "requests": N, "frames": int(r["frames"].sum())}
    batched = Server(codes, policy="batched", msg="fp16", budget_bytes=args.serve_budget,
                     max_inflight=args.serve_inflight)
    plain = Server(codes, policy="plain", budget_bytes=args.serve_budget)
    for staged in (False, True):
        leg = {"llr_source": "pinned host memory, FP16, one copy per launch inside the latency" if staged
               else "device memory (resident before arrival)"}
        # warm-up, then saturation: everything arrives at 0
        batched.run(stream_at(None, min(N, 2000), staged))
        plain.run(stream_at(None, 200, staged))
        sat = batched.run(stream_at(None, N, staged))
        sat_rate = N / sat["makespan"]
        npl = min(N, args.serve_plain_requests)
        psat = plain.run(stream_at(None, npl, staged))
        psat_rate = npl / psat["makespan"]
        leg["saturated"] = {"batched_fp16": {"req_s": sat_rate, **summary(sat, N)},
                            "plain_fp32": {"req_s": psat_rate, **summary(psat, npl)}}
        log(f"serving ({'staged' if staged else 'resident'}) saturated: batched {sat_rate:.0f} req/s "
            f"{leg['saturated']['batched_fp16']['gbit_s']:.2f} Gbit/s; plain {psat_rate:.0f} req/s "
            f"{leg['saturated']['plain_fp32']['gbit_s']:.2f} Gbit/s")
        leg["loads"] = []
        for load in (0.5, 0.8):
            b = batched.run(stream_at(load * sat_rate, N, staged))
            p = plain.run(stream_at(load * psat_rate, npl, staged))
            row = {"load": load, "batched_fp16": {"offered_req_s": load * sat_rate, **summary(b, N)},
                   "plain_fp32": {"offered_req_s": load * psat_rate, **summary(p, npl)}}
            log(f"serving ({'staged' if staged else 'resident'}) load {load}: batched p50 {b['p50_ms']:.2f} "
                f"p99 {b['p99_ms']:.2f} ms; plain (own load) p50 {p['p50_ms']:.2f} p99 {p['p99_ms']:.2f} ms")
            leg["loads"].append(row)
        # the per-request policy at the batched server's half load
        nq = min(N, args.serve_plain_requests // 2)
        q = plain.run(stream_at(0.5 * sat_rate, nq, staged))
        leg["plain_fp32_at_batched_half_load"] = {"offered_req_s": 0.5 * sat_rate, **summary(q, nq)}
        # matched FER: outputs of both policies on the same requests (untimed)
        nv = min(N, args.serve_verify)
        vb = batched.run(stream_at(None, nv, staged), keep_results=True)
        vp = plain.run(stream_at(None, nv, staged), keep_results=True)
        leg["fer_batched_fp16"] = fer(vb["results"], nv)
        leg["fer_plain_fp32"] = fer(vp["results"], nv)
        out["staged_fp16_host" if staged else "device_resident"] = leg
    del host, buf
    for c in codes:
        c.close()
    return out


def calibrate_valu(torch, dev):
    """Lane-operations per second of the VALU probes (libndgsbp_probe.so):
    FMA with 8 and 16 independent chains per lane, add (16), exp2+log2 and
    reciprocal (8), and a mix of 16 FMA and 4 exp2+log2 chains; the best of
    three launches of 2048 x 256 threads each, per CU-cycle at the 2.4 GHz
    peak clock. For the mix: its time per loop trip against the FMA-only and
    transcendental-only times of the same work (additive if the two kinds
    share the issue slots)."""
    import ctypes
    from paper_1202_1060_amd import build
    lib = ctypes.CDLL(build.PROBE_OUT)
    lib.ndgsbp_probe_valu.restype = ctypes.c_int
    lib.ndgsbp_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)]
    blocks = 2048
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    res = {}
    kinds = ((0, "fma_8", 100000), (3, "fma_16", 50000), (4, "add_16", 50000), (1, "exp2_log2_8", 50000),
             (2, "rcp_8", 100000), (5, "mix_fma16_trans8", 40000))
    for kind, name, iters in kinds:
        best = None
        for _ in range(3):
            ms, ops = ctypes.c_float(), ctypes.c_double()
            rc = lib.ndgsbp_probe_valu(kind, blocks, iters, ctypes.c_void_p(out.data_ptr()),
                                       ctypes.byref(ms), ctypes.byref(ops))
            if rc != 0:
                raise RuntimeError(f"probe {name} failed: hip error {rc}")
            if best is None or ms.value < best[0]:
                best = (ms.value, ops.value)
        ms, ops = best
        res[name] = {"ms": ms, "lane_ops": ops, "lane_ops_per_s": ops / (ms * 1e-3),
                     "per_cu_cycle_at_2_4ghz": ops / (ms * 1e-3) / (256 * 2.4e9)}
    # seconds per lane-op of each kind, and the mix against the sum of its parts
    t_fma = 1.0 / res["fma_16"]["lane_ops_per_s"]
    t_trans = 1.0 / res["exp2_log2_8"]["lane_ops_per_s"]
    mix_ops = res["mix_fma16_trans8"]["lane_ops"]
    fma_part, trans_part = mix_ops * 16 / 24, mix_ops * 8 / 24
    additive = fma_part * t_fma + trans_part * t_trans
    res["mix_vs_additive"] = res["mix_fma16_trans8"]["ms"] * 1e-3 / additive
    res["trans_vs_fma"] = res["exp2_log2_8"]["lane_ops_per_s"] / res["fma_16"]["lane_ops_per_s"]
    return {"calibrate_valu": res, "threads": blocks * 256}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--msg", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--frames-per-snr", type=int, default=16384)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target duration of the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fixed", action="store_true", help="skip the fixed-iteration pass")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-message pass")
    ap.add_argument("--lanes", type=int, default=0, choices=[0, 1, 2, 4],
                    help="lanes per CN visit for every message format (0: built-in choice)")
    ap.add_argument("--no-batched", action="store_true", help="skip the mixed-batch leg")
    ap.add_argument("--no-pcie", action="store_true", help="skip the end-to-end (host memory) timing")
    ap.add_argument("--no-schedules", action="store_true",
                    help="skip the flooding, GSBP and vertical-GSBP baselines")
    ap.add_argument("--batch-steps", type=int, default=6)
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (default: user cache dir)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-hbm", action="store_true", help="skip the HBM-tier leg")
    ap.add_argument("--hbm-steps", type=int, default=3)
    ap.add_argument("--hbm-big-frames", type=int, default=131072,
                    help="frames of the n=16896 HBM-tier leg (512 per 64-slot tile and CU: the tile's "
                         "tail, when its last frames run with idle slots, is amortised over 8 refills)")
    ap.add_argument("--serve-requests", type=int, default=30000)
    ap.add_argument("--serve-plain-requests", type=int, default=3000)
    ap.add_argument("--serve-verify", type=int, default=2000)
    ap.add_argument("--serve-pool", type=int, default=1024)
    ap.add_argument("--serve-budget", type=int, default=2 << 30)
    ap.add_argument("--serve-inflight", type=int, default=4)
    ap.add_argument("--calibrate-valu", action="store_true",
                    help="only run the VALU issue-rate probes (FMA, exp2+log2, reciprocal)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the decoder has no multi-GPU path in this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1202_1060_amd as nd
    from ldpcgen import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_valu:
        print(json.dumps(calibrate_valu(torch, dev)), flush=True)
        return
    if args.calibrate_copy:
        # one device-to-device copy of 1 GiB: the counters of this dispatch read
        # 1 GiB fetched and 1 GiB written
        x = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": x.numel() * 4}), flush=True)
        return
    rec = W.SWEEP
    code = W.CODES[rec["code"]]()
    enc = W.encoder_for(rec["code"])
    t0 = time.perf_counter()
    llr_np, cw_np = make_inputs(rec, args.frames_per_snr)
    log(f"inputs: {llr_np.shape} in {time.perf_counter() - t0:.1f} s")
    F = llr_np.shape[0]
    dcode = nd.Code(code, windows=rec["windows"])
    if args.lanes:
        for m in ("fp32", "fp16", "bf16"):
            dcode.tune(m, args.lanes)
    e_iter = dcode.info["edge_updates"]
    llr = torch.from_numpy(llr_np).to(dev)
    out = dict(hard=torch.empty((F, code.n), dtype=torch.uint8, device=dev),
               post=torch.empty((F, code.n), dtype=torch.float32, device=dev),
               iters=torch.empty((F,), dtype=torch.int32, device=dev),
               syn_ok=torch.empty((F,), dtype=torch.uint8, device=dev))
    stream = torch.cuda.current_stream(dev)

    def run(steps, early_stop, msg, dc):
        evs = []
        for _ in range(steps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            nd.decode(dc, llr, rec["max_iter"], early_stop=early_stop, msg=msg, out=out, stream=stream)
            b.record(stream)
            evs.append((a, b))
        return evs

    def measure(steps, early_stop, msg, dc=dcode):
        run(args.warmup, early_stop, msg, dc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs = run(steps, early_stop, msg, dc)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        kern_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        return wall, kern_ms, out["iters"].cpu().numpy(), out["hard"].cpu().numpy()

    def fer_table(iters, hard):
        rows = []
        for i, eb in enumerate(rec["ebn0"]):
            sl = slice(i * args.frames_per_snr, (i + 1) * args.frames_per_snr)
            errs = np.any(hard[sl] != cw_np[sl], axis=1)
            rows.append(dict(ebn0=eb, fer=float(errs.mean()), frame_errors=int(errs.sum()),
                             mean_iters=float(iters[sl].mean())))
        return rows

    bits = F * enc.k
    wall, kern_ms, iters, hard = measure(args.steps, True, args.msg)
    edge_updates = float(iters.astype(np.int64).sum()) * e_iter
    achieved = edge_updates * SLOTS_PER_EDGE_UPDATE / (kern_ms * 1e-3)
    result = {
        "metric": METRIC, "value": round(bits / wall / 1e9, 4), "unit": "Gbit/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.msg == "fp32" else f"f32 compute, {args.msg} messages",
        "data": "synthetic",
        "config": {"workload": "NDGSBP, (3,6)-regular n=2304 code, 8 CN windows of 160 with 16 overlap "
                               "(wrap), Eb/N0 1.0-2.5 dB step 0.25 x 16384 frames, I_max 20, "
                               "syndrome stop",
                   "frames_per_step": F, "k_info": enc.k, "n": code.n, "max_iter": rec["max_iter"],
                   "early_stop": True, "msg": args.msg,
                   "lanes_per_cn": dcode.info[f"lanes_{args.msg}"]},
        "edge_updates_per_s": edge_updates / (kern_ms * 1e-3),
        "mean_iters": float(iters.mean()),
        "kernel_ms": kern_ms,
        "fer": fer_table(iters, hard),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS_PER_S / 1e12,
                     "unit": "T VALU-slots/s", "frac": achieved / PEAK_SLOTS_PER_S,
                     "traffic": measured_traffic(args.msg),
                     "slots_per_edge_update": SLOTS_PER_EDGE_UPDATE,
                     "frac_of_measured_issue_rates": edge_updates / (kern_ms * 1e-3)
                     / EDGE_UPDATES_PER_S_MEASURED_BOUND},
    }
    if not args.no_fixed:
        fwall, fk, _, _ = measure(max(1, args.steps // 2), False, args.msg)
        fe = F * rec["max_iter"] * e_iter
        result["fixed_iterations"] = {
            "gbit_s": bits / fwall / 1e9, "kernel_ms": fk,
            "edge_updates_per_s": fe / (fk * 1e-3),
            "roofline_frac": fe * SLOTS_PER_EDGE_UPDATE / (fk * 1e-3) / PEAK_SLOTS_PER_S}
    if not args.no_pcie:
        # end to end from host memory: pinned LLRs in, decode, hard decisions
        # back to pinned host memory (for context; `value` keeps the inputs
        # resident in HBM)
        host_llr = torch.from_numpy(llr_np).pin_memory()
        host_hard = torch.empty((F, code.n), dtype=torch.uint8).pin_memory()
        walls = []
        for rep in range(args.warmup + 3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            llr.copy_(host_llr, non_blocking=True)
            nd.decode(dcode, llr, rec["max_iter"], early_stop=True, msg=args.msg, out=out, stream=stream)
            host_hard.copy_(out["hard"], non_blocking=True)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                walls.append(time.perf_counter() - t0)
        pw = float(np.median(walls))
        result["end_to_end_pcie"] = {"gbit_s": bits / pw / 1e9, "ms": pw * 1e3,
                                     "h2d_bytes": int(llr_np.nbytes), "d2h_bytes": int(F * code.n)}
        del host_llr, host_hard
    if args.msg == "fp32" and not args.no_fp16:
        # the precision form: FP16-stored messages, FP32 arithmetic, same frames
        hwall, hk, hiters, hhard = measure(args.steps, True, "fp16")
        result["fp16_messages"] = {"gbit_s": bits / hwall / 1e9, "kernel_ms": hk,
                                   "lanes_per_cn": dcode.info["lanes_fp16"],
                                   "mean_iters": float(hiters.mean()), "fer": fer_table(hiters, hhard)}
    if not args.no_schedules:
        # the same frames under the baseline schedules: flooding BP, GSBP
        # (8 disjoint CN windows) and vertical GSBP (8 VN windows), FP32
        sched = {}
        vn_windows = [np.arange((g * code.n) // 8, ((g + 1) * code.n) // 8, dtype=np.int32) for g in range(8)]
        for name, kw in (("flooding", dict(windows=(1, 0, 1))), ("gsbp", dict(windows=(8, 0, 1))),
                         ("vertical_gsbp", dict(vn_groups=vn_windows))):
            c2 = nd.Code(code, **kw)
            w2, k2, it2, h2 = measure(max(1, args.steps // 2), True, "fp32", c2)
            sched[name] = {"gbit_s": bits / w2 / 1e9, "kernel_ms": k2, "mean_iters": float(it2.mean()),
                           "cn_visits_per_iter": c2.info["cn_visits"],
                           "edge_updates_per_iter": c2.info["edge_updates"],
                           "frame_errors": int(sum(r["frame_errors"] for r in fer_table(it2, h2))),
                           "fer": fer_table(it2, h2)}
            log(f"schedule {name}: {sched[name]['gbit_s']:.2f} Gbit/s, mean iters {sched[name]['mean_iters']:.2f}, "
                f"frame errors {sched[name]['frame_errors']}")
            c2.close()
        result["schedules"] = sched
    if not args.no_batched:
        result["batched"] = bench_batched(args, torch, nd, W, dev, log)
    if not args.no_hbm:
        result["hbm_tier"] = bench_hbm(args, torch, nd, W, dev, log, llr_np, enc.k)
    if not args.no_serving:
        result["serving"] = bench_serving(args, torch, nd, W, dev, log)
    if not args.no_cpu_baseline:
        import oracle
        groups = oracle.windows(code.m, *rec["windows"][:2], bool(rec["windows"][2]))
        result["cpu_baseline"] = cpu_baseline(code, groups, llr_np, rec, args.frames_per_snr,
                                              args.cpu_seconds, enc.k, gpu_hard=hard)
    dcode.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
