"""Pure-Python NDGSBP schedule on tiny graphs, over a pluggable algebra.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One schedule (Initialization and Steps 2-4 of Sec. II-C) runs over either
* ``RealAlgebra``: messages are FP64 LLRs; the CN update is eq. (1) written
  literally as 2 atanh(prod tanh(x/2)) (no clamp) and the VN update eq. (2);
* ``ReachAlgebra``: a message is the set of VN indices whose channel value
  it depends on. The CN update is the union over N(m)\\n and the VN update is
  {n} united with the union over M(n)\\m. This is the bookkeeping the paper
  uses when it lists, for its Fig. 1 example, which channel messages each VN
  has received after each sub-iteration (Sec. II-A).
"""
from __future__ import annotations

import math


class RealAlgebra:
    zero_cv = 0.0

    def __init__(self, lch):
        self.lch = [float(x) for x in lch]

    def init_vc(self, n):
        return self.lch[n]

    def cn(self, incoming):
        # eq. (1)
        p = 1.0
        for x in incoming:
            p *= math.tanh(0.5 * x)
        return 2.0 * math.atanh(p)

    def vn(self, n, incoming):
        # eq. (2)
        return self.lch[n] + math.fsum(incoming)

    def total(self, n, incoming):
        # eq. (3)
        return self.lch[n] + math.fsum(incoming)


class ReachAlgebra:
    zero_cv = frozenset()

    def init_vc(self, n):
        return frozenset([n])

    def cn(self, incoming):
        out = frozenset()
        for s in incoming:
            out = out | s
        return out

    def vn(self, n, incoming):
        out = frozenset([n])
        for s in incoming:
            out = out | s
        return out

    def total(self, n, incoming):
        return self.vn(n, incoming)


def run(rows, n, groups, n_iter, algebra, early_stop=False, trace=None, groups_per_iteration=0):
    """rows[m] = N(m) (VN ids); groups = ordered list of CN-id lists; with
    groups_per_iteration = Gp > 0, iteration it (from 1) takes the groups
    of block (it - 1) mod (len(groups) / Gp), Gp groups per block.

    ``trace``, if a list, receives after every sub-iteration a dict
    {vn: union (or list) of the CN->VN messages it currently holds}.
    Returns (totals, hard, iters, syndrome_ok); hard/syndrome only for reals."""
    cols = [[] for _ in range(n)]
    for m, r in enumerate(rows):
        for v in r:
            cols[v].append(m)
    lcv = {(m, v): algebra.zero_cv for m, r in enumerate(rows) for v in r}
    lvc = {(m, v): algebra.init_vc(v) for m, r in enumerate(rows) for v in r}
    real = isinstance(algebra, RealAlgebra)
    totals = hard = None
    ok = False
    used = n_iter
    gp = groups_per_iteration or len(groups)
    blocks = [groups[b:b + gp] for b in range(0, len(groups), gp)]
    for it in range(1, n_iter + 1):
        for grp in blocks[(it - 1) % len(blocks)]:
            # (a) CN update: every CN of the group reads the pre-group lvc
            new = {}
            for m in grp:
                for v in rows[m]:
                    new[(m, v)] = algebra.cn([lvc[(m, u)] for u in rows[m] if u != v])
            lcv.update(new)
            # (b) VN update for every VN touched by the group, all of its edges
            touched = sorted({v for m in grp for v in rows[m]})
            for v in touched:
                for m in cols[v]:
                    lvc[(m, v)] = algebra.vn(v, [lcv[(mm, v)] for mm in cols[v] if mm != m])
            if trace is not None:
                if real:
                    trace.append({v: [lcv[(m, v)] for m in cols[v]] for v in range(n)})
                else:
                    trace.append({v: algebra.cn([lcv[(m, v)] for m in cols[v]]) for v in range(n)})
        totals = [algebra.total(v, [lcv[(m, v)] for m in cols[v]]) for v in range(n)]
        if real:
            hard = [1 if t < 0.0 else 0 for t in totals]
            ok = all(sum(hard[v] for v in r) % 2 == 0 for r in rows)
            if early_stop and ok:
                used = it
                break
    return totals, hard, used, ok
