"""The seeded workloads: codes, windows and frame streams.

Seeds: code seed 1000+k and frame seed 2000+100k+i for workload k and
Eb/N0 point i. Windows are given as (G, overlap, wrap): window g starts at
floor(g*M/G) and runs to the next start plus ``overlap`` CNs, indices
taken mod M when ``wrap`` is set.
"""
from __future__ import annotations

import functools

import numpy as np

from .codes import regular_code, qc_code, base_mask
from .gf2 import SystematicEncoder
from .channel import make_frames


@functools.lru_cache(maxsize=None)
def code_n96():
    """(3,6)-regular, n=96, m=48, 4-cycle-free (configuration model)."""
    return regular_code(96, 3, 6, seed=1000, girth6=True)


@functools.lru_cache(maxsize=None)
def code_n2304():
    """(3,6)-regular, n=2304, m=1152, 4-cycle-free (configuration model)."""
    return regular_code(2304, 3, 6, seed=1001, girth6=True)


@functools.lru_cache(maxsize=None)
def code_qc(n: int, rate: str, seed: int):
    """Quasi-cyclic code from a 24-column base matrix, z = n/24."""
    assert n % 24 == 0
    z = n // 24
    return qc_code(base_mask(rate, seed), z, seed)


@functools.lru_cache(maxsize=None)
def encoder_for(code_key):
    return SystematicEncoder(CODES[code_key]())


@functools.lru_cache(maxsize=None)
def code_n504():
    """(3,6)-regular, n=504, m=252, 4-cycle-free: stand-in for MacKay's (504,252)."""
    return regular_code(504, 3, 6, seed=1040, girth6=True)


@functools.lru_cache(maxsize=None)
def code_n816():
    """(4,6)-regular, n=816, m=544, 4-cycle-free: stand-in for MacKay's (816,*) code."""
    return regular_code(816, 4, 6, seed=1041, girth6=True)


CODES = {
    "n96": code_n96,
    "n2304": code_n2304,
    "n504": code_n504,
    "n816": code_n816,
    "qc2304": lambda: code_qc(2304, "1/2", 1002),
}

# QC codes of the batched workload: one per (length, rate), seeds 1003..1014
BATCH_N = (576, 1152, 2304, 4608)
BATCH_RATES = ("1/2", "2/3", "3/4")


def qc_key(n: int, rate: str) -> str:
    return f"qc{n}r{rate.replace('/', '_')}"


for _i, (_n, _r) in enumerate((n, r) for n in BATCH_N for r in BATCH_RATES):
    CODES[qc_key(_n, _r)] = functools.partial(code_qc, _n, _r, 1003 + _i)

# resident codes of the serving workload, seeds 1020..1022
SERVE_CODES = ((648, "5/6"), (1944, "1/2"), (8064, "1/2"))
for _i, (_n, _r) in enumerate(SERVE_CODES):
    CODES[qc_key(_n, _r)] = functools.partial(code_qc, _n, _r, 1020 + _i)


def base_rows(rate: str) -> int:
    from .codes import QC_PROFILES
    return QC_PROFILES[rate]["mb"]

# workload recipes
SMALL = dict(name="ndgsbp-n96-w4o2", code="n96", windows=(4, 2, 1), max_iter=10,
             early_stop=False, ebn0=[2.0], frames=200, all_zero=True, seed=2000)
SWEEP = dict(name="ndgsbp-n2304-w8o16", code="n2304", windows=(8, 16, 1), max_iter=20,
             early_stop=True, ebn0=[1.0, 1.25, 1.5, 1.75, 2.0, 2.25, 2.5], frames=16384,
             all_zero=False, seed=2100)
SWEEP_FLOODING = dict(SWEEP, name="flooding-n2304", windows=(1, 0, 1))
SWEEP_GSBP = dict(SWEEP, name="gsbp-n2304-w8", windows=(8, 0, 1))
PRECISION = dict(name="ndgsbp-qc2304-w12o24", code="qc2304", windows=(12, 24, 1), max_iter=15,
                 early_stop=True, ebn0=[1.5, 2.0], frames=65536, all_zero=False, seed=2200)


# Batched decoding: 256 problems, each a QC code of length in BATCH_N and
# rate in BATCH_RATES (z = n/24), 64..1024 frames (log-uniform), Eb/N0 in
# [1, 3] dB, 6..16 CN windows with overlap z/4 (wrap), FP16 messages,
# 20 iterations, syndrome stop.
BATCH = dict(name="batched-qc-mixed-256", problems=256, frames=(64, 1024), ebn0=(1.0, 3.0),
             groups=(6, 16), max_iter=20, early_stop=True, msg="fp16", seed=2300)

# Serving: requests over the three SERVE_CODES (one base row per window,
# overlap floor(z/4), wrap), 1..512 frames (geometric, mean 32), Eb/N0 in
# [1.5, 3.5] dB, Poisson arrivals, FP16 messages, 20 iterations, syndrome stop.
SERVE = dict(name="serving-qc-3codes", mean_frames=32, max_frames=512, ebn0=(1.5, 3.5),
             max_iter=20, early_stop=True, msg="fp16", seed=2400)


def _philox(*key):
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(k) for k in key])))


def batch_problems(recipe: dict = BATCH, count: int | None = None):
    """The problem list of the batched workload (no frames yet): dicts with
    code key, n, rate, windows (G, o, 1), frames, Eb/N0 and frame seed."""
    rng = _philox(recipe["seed"], 0)
    out = []
    lo, hi = recipe["frames"]
    for i in range(recipe["problems"] if count is None else count):
        n = int(BATCH_N[rng.integers(len(BATCH_N))])
        rate = BATCH_RATES[rng.integers(len(BATCH_RATES))]
        z = n // 24
        G = int(rng.integers(recipe["groups"][0], recipe["groups"][1] + 1))
        F = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))
        eb = float(rng.uniform(*recipe["ebn0"]))
        out.append(dict(index=i, code=qc_key(n, rate), n=n, rate=rate, windows=(G, z // 4, 1),
                        frames=F, ebn0=eb, max_iter=recipe["max_iter"],
                        seed=recipe["seed"] * 1000 + 1 + i))
    return out


def serve_windows(n: int, rate: str):
    """One base row per window, overlap floor(z/4), wrap."""
    return (base_rows(rate), (n // 24) // 4, 1)


SERVE_BINS = np.round(np.arange(1.5, 3.5 + 1e-9, 0.25), 2)  # Eb/N0 grid of the frame pools


def serve_requests(recipe: dict = SERVE, count: int = 256):
    """Request stream of the serving workload at unit offered load (one
    request per second on average; scale ``arrival`` by 1/rate). Arrays:
    arrival (Poisson process), code (index into SERVE_CODES), frames
    (geometric, mean 32, at most 512), ebn0 (uniform), bin (nearest point of
    SERVE_BINS) and pool offset (uniform, so the request's frames are pool
    frames offset .. offset + frames - 1 of its code and bin)."""
    rng = _philox(recipe["seed"], 0)
    arrival = np.cumsum(rng.exponential(1.0, size=count))
    code = rng.integers(len(SERVE_CODES), size=count)
    frames = np.minimum(recipe["max_frames"], rng.geometric(1.0 / recipe["mean_frames"], size=count))
    ebn0 = rng.uniform(*recipe["ebn0"], size=count)
    b = np.clip(np.round((ebn0 - SERVE_BINS[0]) / 0.25).astype(np.int64), 0, len(SERVE_BINS) - 1)
    u = rng.random(count)
    return dict(arrival=arrival, code=code, frames=frames.astype(np.int64), ebn0=ebn0, bin=b, u=u)


def serve_pool(code_index: int, frames_per_bin: int, recipe: dict = SERVE):
    """Frame pool of one serving code: LLRs (bins, frames_per_bin, n) and
    codewords, random information bits, one seeded stream per bin."""
    n, rate = SERVE_CODES[code_index]
    key = qc_key(n, rate)
    enc = encoder_for(key)
    llr = np.empty((len(SERVE_BINS), frames_per_bin, n), dtype=np.float32)
    cw = np.empty((len(SERVE_BINS), frames_per_bin, n), dtype=np.uint8)
    for i, eb in enumerate(SERVE_BINS):
        llr[i], cw[i] = make_frames(n, frames_per_bin, float(eb), enc.rate,
                                    recipe["seed"] * 1000 + 100 * code_index + i, encoder=enc)
    return llr, cw


def serve_symbols(code_index: int, pool: int, recipe: dict = SERVE):
    """Channel pool of one serving code for requests at any Eb/N0: ``pool``
    codewords of random information bits (uint8 (pool, n)) and unit-variance
    Gaussian noise (float32 (pool, n)), seeded per code. A frame drawn from
    pool row j at noise level sigma has LLRs (2 / sigma^2) (x + sigma w) with
    x = 1 - 2 c (BPSK)."""
    n, rate = SERVE_CODES[code_index]
    enc = encoder_for(qc_key(n, rate))
    rng = _philox(recipe["seed"], 1, code_index)
    u = rng.integers(0, 2, size=(pool, enc.k), dtype=np.uint8)
    cw = enc.encode(u)
    w = rng.standard_normal((pool, n), dtype=np.float32)
    return cw, w


def problem_frames(prob: dict, num_frames: int | None = None):
    """LLRs and codewords of a batched problem or a serving request."""
    enc = encoder_for(prob["code"])
    nf = prob["frames"] if num_frames is None else num_frames
    return make_frames(prob["n"], nf, prob["ebn0"], enc.rate, prob["seed"], encoder=enc)


def frames(recipe: dict, snr_index: int, num_frames: int | None = None, first_frame: int = 0):
    """LLRs and codewords for one Eb/N0 point of a recipe."""
    code = CODES[recipe["code"]]()
    enc = encoder_for(recipe["code"])
    nf = recipe["frames"] if num_frames is None else num_frames
    seed = recipe["seed"] + snr_index
    return make_frames(code.n, nf, recipe["ebn0"][snr_index], enc.rate, seed,
                       encoder=None if recipe["all_zero"] else enc, first_frame=first_frame)
