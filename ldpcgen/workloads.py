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


CODES = {
    "n96": code_n96,
    "n2304": code_n2304,
    "qc2304": lambda: code_qc(2304, "1/2", 1002),
}

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


def frames(recipe: dict, snr_index: int, num_frames: int | None = None, first_frame: int = 0):
    """LLRs and codewords for one Eb/N0 point of a recipe."""
    code = CODES[recipe["code"]]()
    enc = encoder_for(recipe["code"])
    nf = recipe["frames"] if num_frames is None else num_frames
    seed = recipe["seed"] + snr_index
    return make_frames(code.n, nf, recipe["ebn0"][snr_index], enc.rate, seed,
                       encoder=None if recipe["all_zero"] else enc, first_frame=first_frame)
