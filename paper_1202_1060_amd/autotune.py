"""Launch-option autotuner for batched decoding and single-code decodes.

It times candidate launch choices on the caller's own problems (HIP events
on one stream, after a warm-up launch) and keeps the fastest. The choices:

* CN-lane mapping: one lane per CN visit, or two or four lanes sharing it
  (``lanes_per_cn``), or each code's own choice, which the tuner first sets
  per code and grouping by timing it alone (``tune_lanes_per_code``);
* launch classes: one persistent launch per kernel variant, or one per
  variant and power-of-two LDS size (``split_by_size``), which sizes each
  launch's workgroups and LDS to its problems;
* workgroup size cap (``max_threads``): fewer lanes per group means more
  workgroups (frames) resident per compute unit, more visits per lane;
* streams the launch classes are spread over, so the tail of one persistent
  launch overlaps the next.

Results are cached in a JSON file keyed by the problem signature (code
sizes, groupings, frame counts rounded to powers of two), message format,
stop rule and device name. Every candidate runs the same decoder: only the
time differs, never the result.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

import torch

from . import Batch, BatchOptions, Problem, Code, decode, new_outputs

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ndgsbp", "autotune.json")


def _cache_path(path):
    return path or os.environ.get("NDGSBP_TUNE_CACHE") or DEFAULT_CACHE


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, db):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _device_sig(dev) -> list:
    """Identity of the device kind a tuning result holds for: the ISA, the
    CU count and the memory size (the marketing name can be empty, e.g.
    under a profiler)."""
    pr = torch.cuda.get_device_properties(dev)
    return [getattr(pr, "gcnArchName", ""), pr.multi_processor_count, pr.total_memory]


def _code_sig(code: Code):
    i = code.info
    return (i["m"], i["n"], i["nnz"], i["num_groups"], i["cn_visits"], i["edge_updates"],
            i["max_cn_degree"])


def batch_signature(problems, msg: str, early_stop: bool) -> str:
    items = sorted((_code_sig(p.code), int(p.llr.shape[0]).bit_length(), p.max_iter) for p in problems)
    dev = problems[0].llr.device if problems else torch.device("cuda", 0)
    blob = json.dumps([items, msg, bool(early_stop), _device_sig(dev)])
    return "batch:" + hashlib.sha1(blob.encode()).hexdigest()


def batch_candidates():
    for lanes, split, threads, streams in itertools.product((0, 1, 2), (1, 0), (0, 512, 256),
                                                            (4, 1)):
        yield BatchOptions(lanes, split, threads, streams)


def _time_launches(fn, reps, stream):
    fn()
    torch.cuda.synchronize()
    evs = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        evs.append((a, b))
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in evs)
    return ts[len(ts) // 2]


def tune_lanes_per_code(problems, *, msg: str = "fp16", early_stop: bool = True, reps: int = 3,
                        min_frames: int = 8192, log=None):
    """For each set of problems that share a code and grouping: time that
    set alone (its frames repeated up to about ``min_frames``, so that the
    launch runs in steady state rather than in its tail) with 1, 2 and 4
    lanes per CN visit, and tune the set's codes (ldpc_code_tune) to the
    fastest. Returns {code signature: lanes}."""
    sets = {}
    for p in problems:
        sets.setdefault(_code_sig(p.code), []).append(p)
    dev = problems[0].llr.device
    stream = torch.cuda.current_stream(dev)
    chosen = {}
    for sig, ps in sets.items():
        frames = sum(int(p.llr.shape[0]) for p in ps)
        if frames == 0:
            continue
        rep = max(1, -(-min_frames // frames))
        llr = torch.cat([p.llr for p in ps] * rep)
        code = ps[0].code
        best = None
        for lanes in (1, 2, 4):
            try:
                code.tune(msg, lanes)
            except Exception:  # no kernel variant with that mapping
                continue
            b = Batch([Problem(code, llr, max(p.max_iter for p in ps), want_post=False)], msg=msg,
                      early_stop=early_stop, options=BatchOptions(0, 1, 512, 1))
            ms = _time_launches(lambda: b.launch(stream), reps, stream)
            b.close()
            if best is None or ms < best[0]:
                best = (ms, lanes)
        for p in ps:
            p.code.tune(msg, best[1])
        chosen[sig] = best[1]
        if log:
            log(f"autotune lanes {sig[:2]} x{len(ps)}: {best[1]} ({best[0]:.3f} ms)")
    return chosen


def tune_batch(problems, *, msg: str = "fp16", early_stop: bool = True, reps: int = 3,
               cache: str | None = None, candidates=None, force: bool = False, per_code_lanes: bool = True,
               log=None):
    """Fastest BatchOptions for these problems (cached). With
    ``per_code_lanes`` the codes are first tuned set by set
    (tune_lanes_per_code), which the candidates with lanes_per_cn = 0 use;
    the codes keep those mappings only if such a candidate wins. Candidates
    that a code cannot take (e.g. two lanes where its variant has none) are
    skipped."""
    path = _cache_path(cache)
    key = batch_signature(problems, msg, early_stop)
    db = _load(path)
    if not force and key in db:
        lanes = {tuple(k): v for k, v in db[key].get("code_lanes", [])}
        for p in problems:
            if _code_sig(p.code) in lanes:
                p.code.tune(msg, lanes[_code_sig(p.code)])
        return BatchOptions.from_tuple(db[key]["options"])
    dev = problems[0].llr.device
    stream = torch.cuda.current_stream(dev)
    field = "lanes_" + msg
    before = [p.code.info[field] for p in problems]
    chosen = tune_lanes_per_code(problems, msg=msg, early_stop=early_stop, reps=reps, log=log) \
        if per_code_lanes else {}
    results = []
    for opt in (candidates or batch_candidates()):
        try:
            b = Batch(problems, msg=msg, early_stop=early_stop, options=opt)
        except Exception as e:  # an option the codes cannot take
            if log:
                log(f"autotune skip {opt}: {e}")
            continue
        ms = _time_launches(lambda: b.launch(stream), reps, stream)
        if log:
            log(f"autotune {opt} launches={b.info['num_launches']}: {ms:.3f} ms")
        b.close()
        results.append((ms, opt))
    if not results:
        raise RuntimeError("no launch option worked for this batch")
    ms, best = min(results, key=lambda r: r[0])
    if best.lanes_per_cn != 0 and chosen:
        # the per-code mappings lost: give the codes back their own
        for p, lanes in zip(problems, before):
            p.code.tune(msg, lanes)
        chosen = {}
    db = _load(path)
    db[key] = dict(options=list(best.as_tuple()), ms=ms, tried=len(results), when=time.time(),
                   code_lanes=[[list(k), v] for k, v in chosen.items()])
    _store(path, db)
    return best


def tune_code(code: Code, llr: torch.Tensor, max_iter: int, *, msg: str = "fp32",
              early_stop: bool = True, reps: int = 3, cache: str | None = None,
              force: bool = False, log=None) -> int:
    """Pick the faster CN-lane mapping of one code for ``msg`` on sample
    frames ``llr``, apply it (ldpc_code_tune) and return it."""
    path = _cache_path(cache)
    blob = json.dumps([_code_sig(code), int(llr.shape[0]).bit_length(), max_iter, msg, bool(early_stop),
                       _device_sig(llr.device)])
    key = "code:" + hashlib.sha1(blob.encode()).hexdigest()
    db = _load(path)
    if not force and key in db:
        code.tune(msg, db[key]["lanes"])
        return db[key]["lanes"]
    stream = torch.cuda.current_stream(llr.device)
    out = new_outputs(int(llr.shape[0]), code.n, llr.device, want_post=False)
    best = None
    for lanes in (1, 2, 4):
        try:
            code.tune(msg, lanes)
        except Exception:
            continue
        ms = _time_launches(lambda: decode(code, llr, max_iter, early_stop=early_stop, msg=msg, out=out,
                                           stream=stream), reps, stream)
        if log:
            log(f"autotune code lanes={lanes}: {ms:.3f} ms")
        if best is None or ms < best[0]:
            best = (ms, lanes)
    code.tune(msg, best[1])
    db = _load(path)
    db[key] = dict(lanes=best[1], ms=best[0], when=time.time())
    _store(path, db)
    return best[1]


__all__ = ["tune_batch", "tune_code", "tune_lanes_per_code", "batch_signature", "batch_candidates",
           "Problem"]
