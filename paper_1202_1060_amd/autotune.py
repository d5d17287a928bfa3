"""Launch-option autotuner for batched decoding and single-code decodes.

It times candidate launch choices on the caller's own problems (HIP events
on one stream, after a warm-up launch) and keeps the fastest. The choices:

* CN-lane mapping: one lane per CN visit, or two lanes sharing it
  (``lanes_per_cn``), or each code's own choice;
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


def _code_sig(code: Code):
    i = code.info
    return (i["m"], i["n"], i["nnz"], i["num_groups"], i["cn_visits"], i["edge_updates"],
            i["max_cn_degree"])


def batch_signature(problems, msg: str, early_stop: bool) -> str:
    items = sorted((_code_sig(p.code), int(p.llr.shape[0]).bit_length(), p.max_iter) for p in problems)
    dev = problems[0].llr.device if problems else torch.device("cuda", 0)
    blob = json.dumps([items, msg, bool(early_stop), torch.cuda.get_device_name(dev)])
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


def tune_batch(problems, *, msg: str = "fp16", early_stop: bool = True, reps: int = 3,
               cache: str | None = None, candidates=None, force: bool = False, log=None):
    """Fastest BatchOptions for these problems (cached). Candidates that a
    code cannot take (e.g. two lanes where its variant has none) are
    skipped."""
    path = _cache_path(cache)
    key = batch_signature(problems, msg, early_stop)
    db = _load(path)
    if not force and key in db:
        return BatchOptions.from_tuple(db[key]["options"])
    dev = problems[0].llr.device
    stream = torch.cuda.current_stream(dev)
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
    db = _load(path)
    db[key] = dict(options=list(best.as_tuple()), ms=ms, tried=len(results), when=time.time())
    _store(path, db)
    return best


def tune_code(code: Code, llr: torch.Tensor, max_iter: int, *, msg: str = "fp32",
              early_stop: bool = True, reps: int = 3, cache: str | None = None,
              force: bool = False, log=None) -> int:
    """Pick the faster CN-lane mapping of one code for ``msg`` on sample
    frames ``llr``, apply it (ldpc_code_tune) and return it."""
    path = _cache_path(cache)
    blob = json.dumps([_code_sig(code), int(llr.shape[0]).bit_length(), max_iter, msg, bool(early_stop),
                       torch.cuda.get_device_name(llr.device)])
    key = "code:" + hashlib.sha1(blob.encode()).hexdigest()
    db = _load(path)
    if not force and key in db:
        code.tune(msg, db[key]["lanes"])
        return db[key]["lanes"]
    stream = torch.cuda.current_stream(llr.device)
    out = new_outputs(int(llr.shape[0]), code.n, llr.device, want_post=False)
    best = None
    for lanes in (1, 2):
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


__all__ = ["tune_batch", "tune_code", "batch_signature", "batch_candidates", "Problem"]
