"""BPSK over AWGN and the channel LLR of Sec. II-C.

Bit c is sent as x = 1 - 2c (0 -> +1), received as y = x + sigma*w with
w ~ N(0, 1), and its LLR is L = 2 y / sigma^2 (Sec. II-C). Eb/N0 maps to
sigma by sigma^2 = 1 / (2 R 10^(EbN0/10)) with R = K/N.

Frames are produced in blocks; block b of a stream draws from its own
Philox stream keyed by (seed, b), so any block range can be regenerated
without the others. LLRs are float32; the oracle widens the same array.
"""
from __future__ import annotations

import math

import numpy as np

BLOCK = 256


def ebn0_to_sigma(ebn0_db: float, rate: float) -> float:
    return math.sqrt(1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0)))


def _gen(seed, block, sub):
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed), int(block), int(sub)])))


def bpsk_awgn_llr(codewords: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """codewords: (F, n) uint8 -> float32 LLRs (F, n)."""
    c = np.asarray(codewords, dtype=np.uint8)
    w = rng.standard_normal(c.shape, dtype=np.float32)
    x = (1.0 - 2.0 * c.astype(np.float32)).astype(np.float32)
    y = x + np.float32(sigma) * w
    return (np.float32(2.0 / (sigma * sigma)) * y).astype(np.float32)


def make_frames(n: int, num_frames: int, ebn0_db: float, rate: float, seed,
                encoder=None, first_frame: int = 0):
    """Frames ``first_frame .. first_frame+num_frames-1`` of the stream.

    With ``encoder`` the codewords carry uniform random information bits
    (encoded systematically); without it the all-zero codeword is sent.
    Returns (llr float32 (F, n), codewords uint8 (F, n))."""
    sigma = ebn0_to_sigma(ebn0_db, rate)
    llr = np.empty((num_frames, n), dtype=np.float32)
    cw = np.zeros((num_frames, n), dtype=np.uint8)
    f0 = first_frame
    f1 = first_frame + num_frames
    b0 = f0 // BLOCK
    b1 = (f1 + BLOCK - 1) // BLOCK
    for b in range(b0, b1):
        lo = max(f0, b * BLOCK)
        hi = min(f1, (b + 1) * BLOCK)
        if encoder is not None:
            ug = _gen(seed, b, 1)
            u = ug.integers(0, 2, size=(BLOCK, encoder.k), dtype=np.uint8)
            cb = encoder.encode(u)
        else:
            cb = np.zeros((BLOCK, n), dtype=np.uint8)
        lb = bpsk_awgn_llr(cb, sigma, _gen(seed, b, 2))
        llr[lo - f0:hi - f0] = lb[lo - b * BLOCK:hi - b * BLOCK]
        cw[lo - f0:hi - f0] = cb[lo - b * BLOCK:hi - b * BLOCK]
    return llr, cw


def device_all_zero_llr(n: int, num_frames: int, ebn0_db: float, rate: float, seed: int, device):
    """All-zero codeword over BPSK/AWGN, generated on a torch device with a
    seeded torch generator: L = (2 / sigma^2) (1 + sigma w). For error-rate
    sweeps whose frame counts make host generation the bottleneck."""
    import torch
    sigma = ebn0_to_sigma(ebn0_db, rate)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    w = torch.randn((num_frames, n), generator=g, device=device, dtype=torch.float32)
    return (w * float(sigma) + 1.0) * float(2.0 / (sigma * sigma))
