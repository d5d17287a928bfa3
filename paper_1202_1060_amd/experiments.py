"""Error rates of BP, GSBP and NDGSBP at equal complexity (Sec. IV setup).

The paper compares, on MacKay's (504,252) (3,6) code with G = 12 and on its
(816,544) (4,6) code with G = 16:

* standard BP (flooding: one group holding every CN), I_max = 1000;
* GSBP (G disjoint CN groups), I_max = 1000;
* NDGSBP (G groups by Step 1 with overlap ratio r = 0.4), with the iteration
  cap lowered to M I_max / (M + (G - 1) N_G r), so that every decoder may
  spend the same number of CN updates;
* NDGSBP with groups that make Step 1's free choices for a large CoCSG
  (``grouping.cocsg_groups``, the open direction of Sec. V), same sizes and
  budget;
* vertical group-shuffled BP (the prior art Sec. I cites: G groups of VNs,
  a random partition), I_max = 1000; every edge message is computed once
  per iteration, as in BP.

MacKay's matrices are not available; seeded (3,6) n=504 and (4,6) n=816
codes with the same sizes stand in for them. Frames carry the all-zero
codeword (the decoders are symmetric), generated on the GPU; every decode
runs the library's kernels with FP32 messages and syndrome stop. BER counts
codeword bits. NDGSBP runs three times: with one Step-1 grouping for the
whole decode, with a fresh Step-1 grouping for every iteration (as Step 4's
return to Step 1 reads), drawn ahead of time up to the iteration cap, and
with a fresh CoCSG-seeking grouping for every iteration. The mean CoCSG of
each schedule is reported.

Usage: python -m paper_1202_1060_amd.experiments [--frames F] [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import Code, decode
from .grouping import (group_size, step1_groups, disjoint_random_groups,
                       equal_complexity_iterations, cocsg, cocsg_groups)

SETUPS = {
    # code key, G, r, I_max of BP and GSBP, grouping seed
    "n504": dict(G=12, r=0.4, I_max=1000, seed=3100),
    "n816": dict(G=16, r=0.4, I_max=1000, seed=3101),
}


def clopper_pearson(k, n, alpha=0.05):
    from scipy.stats import beta
    lo = 0.0 if k == 0 else float(beta.ppf(alpha / 2, k, n - k + 1))
    hi = 1.0 if k == n else float(beta.ppf(1 - alpha / 2, k + 1, n - k))
    return lo, hi


def decoders(code, setup):
    """(name, groups, groups per iteration, iteration cap, CN updates per
    iteration) of the decoders for one code: BP, GSBP, NDGSBP with one
    Step-1 grouping, NDGSBP with a fresh Step-1 grouping for every iteration
    up to its cap (Step 4 returns to Step 1), the same with CoCSG-seeking
    groupings, and vertical GSBP (VN groups)."""
    M = code.m
    G, r, I = setup["G"], setup["r"], setup["I_max"]
    rng = np.random.Generator(np.random.Philox(setup["seed"]))
    N_G = group_size(M, G, r)
    nd_groups = step1_groups(M, G, r, rng, N_G)
    gs_groups = disjoint_random_groups(M, G, rng)
    I_nd = equal_complexity_iterations(M, I, G, N_G, r)
    sched, sched_l = [], []
    ell_step1, ell_cocsg = [], []
    for _ in range(I_nd):
        grp = step1_groups(M, G, r, rng, N_G)
        sched += grp
        ell_step1.append(cocsg(code, grp)[0])
    for _ in range(I_nd):
        grp = cocsg_groups(code, G, r, rng, N_G)
        sched_l += grp
        ell_cocsg.append(cocsg(code, grp)[0])
    per_iter = int(sum(len(g) for g in nd_groups))
    return [("bp", [np.arange(M, dtype=np.int32)], 0, I, M),
            ("gsbp", gs_groups, 0, I, M),
            ("ndgsbp", nd_groups, 0, I_nd, per_iter),
            ("ndgsbp_regroup", sched, G, I_nd, per_iter),
            ("ndgsbp_cocsg_regroup", sched_l, G, I_nd, per_iter),
            ("vgsbp", [np.sort(x).astype(np.int32) for x in np.array_split(rng.permutation(code.n), G)],
             0, I, M)], \
        dict(N_G=N_G, I_ndgsbp=I_nd, ell_gsbp=cocsg(code, gs_groups)[0], ell_step1=float(np.mean(ell_step1)),
             ell_cocsg=float(np.mean(ell_cocsg)))


def run(code_key, ebn0s, frames, device, log=None, chunk=1 << 18, only=None):
    from ldpcgen import workloads as W
    from ldpcgen.channel import device_all_zero_llr
    from ldpcgen.gf2 import gf2_rank
    code = W.CODES[code_key]()
    K = code.n - gf2_rank(code.dense())
    rate = K / code.n
    setup = SETUPS[code_key]
    decs, meta = decoders(code, setup)
    out = dict(code=code_key, n=code.n, m=code.m, k=K, **setup, **meta, points=[])
    for i, eb in enumerate(ebn0s):
        row = dict(ebn0=eb)
        for name, groups, gpi, cap, cn_per_iter in decs:
            if only and name not in only:
                continue
            if name == "vgsbp":  # VN groups: the vertical schedule
                dcode = Code(code, vn_groups=groups, device=device.index or 0)
            else:
                dcode = Code(code, groups=groups, device=device.index or 0, groups_per_iteration=gpi)
            fe = be = it = 0
            t0 = time.perf_counter()
            done = 0
            while done < frames:
                F = min(chunk, frames - done)
                llr = device_all_zero_llr(code.n, F, eb, rate, 7000 + 100 * i + done // chunk, device)
                o = decode(dcode, llr, cap, early_stop=True, want_post=False)
                hard = o["hard"]
                errs = hard.sum(dim=1, dtype=torch.int64)
                fe += int((errs > 0).sum())
                be += int(errs.sum())
                it += int(o["iters"].sum(dtype=torch.int64))
                done += F
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            dcode.close()
            lo, hi = clopper_pearson(fe, frames)
            row[name] = dict(fer=fe / frames, fer_ci95=[lo, hi], frame_errors=fe, ber=be / (frames * code.n),
                             mean_iters=it / frames, cn_updates_per_frame=it / frames * cn_per_iter,
                             iter_cap=cap, seconds=dt)
            if log:
                log(f"{code_key} {eb:.2f} dB {name:7s} FER {fe / frames:.3e} BER {be / (frames * code.n):.3e} "
                    f"iters {it / frames:.2f} ({dt:.1f} s)")
        out["points"].append(row)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--codes", nargs="+", default=["n504", "n816"])
    ap.add_argument("--decoders", nargs="+", default=None, help="subset of the decoders to run")
    ap.add_argument("--ebn0", nargs="+", type=float, default=[1.0, 1.5, 2.0, 2.5, 3.0])
    ap.add_argument("--frames", type=int, default=1 << 20)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    dev = torch.device("cuda", 0)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    res = [run(c, args.ebn0, args.frames, dev, log, only=args.decoders) for c in args.codes]
    text = json.dumps(res, indent=1)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()
