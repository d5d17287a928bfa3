"""Gaussian-approximation (GA) convergence analysis of Sec. III (Table I).

Messages are modelled as consistent Gaussians, so only their means are
tracked (all-zero codeword, BPSK, AWGN). The CN update uses the function
Phi(mu) = 1 - E[tanh(u/2)], u ~ N(mu, 2 mu), evaluated with the published
two-piece approximation of Chung, Richardson and Urbanke (2001):
    Phi(x) = exp(-0.4527 x^0.86 + 0.0218)                for 0 < x < 10,
    Phi(x) = sqrt(pi/x) exp(-x/4) (1 - 10/(7x))          for x >= 10
(the two pieces differ by about 2% at x = 10; the inverse bisects).
"Error-free" is read as the bit error probability of the posterior,
Q(sqrt(mu_total/2)), falling below 1e-6; iterations are counted from 1.

* ``ga_bp``: the standard flooding recursion
  mu_c(l) = sum_j rho_j Phi^-1(1 - (1 - sum_i lambda_i Phi(mu0 + (i-1) mu_c(l-1)))^(j-1)).
* ``ga_group``: a horizontal group-shuffled recursion with G groups and
  overlap ratio 0 <= r < 0.5 (r = 0: GSBP), following the class structure
  of eq. (4)-(17) under these readings (the printed equations are partly
  garbled): in sub-iteration g, a VN edge into the group sees its other
  i - 1 edges as class a (CN not updated yet in this iteration), class d
  (CN updated in an earlier sub-iteration of this iteration, outside the
  overlap) or class b (CN shared with the previous group); the class-d
  fraction counts the g - 1 groups already done ((g - 1)(1 - r) / (G -
  (G - 1) r), where the printed y has g, which would let y + z exceed 1);
  the class-d mean is the mean over the done groups with the class-b /
  class-c proportions of eq. (5); the overlap CNs' output uses the VNs with
  at least one class-d edge (eq. (15) with p >= 1, renormalised); the
  class-a mean is the mean of every CN's latest message after the previous
  iteration (eq. (17) read as that mean: the printed form names only group
  G). With r = 0 this reproduces the paper's GSBP columns of Table I
  exactly for both ensembles (293, 262, 251 and 438, 386, 376); the r = 0.4
  columns come within 1-4% (240, 211, 203 against 240, 208, 196; 373, 335,
  331 against 368, 324, 317): parity unpinned for r > 0, the values are
  reported beside the table, not held to it.
"""
from __future__ import annotations

import math




def phi(x: float) -> float:
    """Phi(mu) = 1 - E[tanh(u/2)], u ~ N(mu, 2 mu) (two-piece approximation)."""
    if x <= 0.0:
        return 1.0
    if x < 10.0:
        return math.exp(-0.4527 * x ** 0.86 + 0.0218)
    return math.sqrt(math.pi / x) * math.exp(-x / 4.0) * (1.0 - 10.0 / (7.0 * x))


def phi_inv(y: float) -> float:
    """Inverse of phi on its decreasing range (bisection; phi(0) = 1)."""
    if y >= 1.0:
        return 0.0
    if y <= 0.0:
        return math.inf
    lo, hi = 0.0, 1.0
    while phi(hi) > y:
        hi *= 2.0
        if hi > 1e12:
            return math.inf
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if phi(mid) > y:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-15 * hi:
            break
    return 0.5 * (lo + hi)


def channel_mean(ebn0_db: float, rate: float) -> float:
    """mu0 = E[2y/sigma^2] = 2/sigma^2 with sigma^2 = 1/(2 R 10^(Eb/N0 / 10))."""
    return 4.0 * rate * 10.0 ** (ebn0_db / 10.0)


def bit_error(mu_total: float) -> float:
    return 0.5 * math.erfc(math.sqrt(max(mu_total, 0.0) / 2.0) / math.sqrt(2.0))


def _cn_mean(mu_v_by_degree, lam, rho):
    """CN-to-VN mean from the VN-to-CN means per VN degree (eq. (15)-(16))."""
    s = sum(lam[i] * phi(mu_v_by_degree[i]) for i in lam)
    return sum(rho[j] * phi_inv(1.0 - (1.0 - s) ** (j - 1)) for j in rho)


def _regular(dv, dc):
    return {dv: 1.0}, {dc: 1.0}


def ga_bp(dv: int, dc: int, rate: float, ebn0_db: float, pe: float = 1e-6, max_iter: int = 100000):
    """Iterations of the flooding GA recursion until the bit error
    probability drops below pe (None if it stalls)."""
    lam, rho = _regular(dv, dc)
    mu0 = channel_mean(ebn0_db, rate)
    muc = 0.0
    for l in range(1, max_iter + 1):
        new = _cn_mean({i: mu0 + (i - 1) * muc for i in lam}, lam, rho)
        if bit_error(mu0 + dv * new) < pe:
            return l
        if abs(new - muc) <= 1e-14 * max(1.0, new):
            return None
        muc = new
    return None


def _mixture(i, p_frac, q_frac, mu_a, mu_d, mu_b, mu0, p_min=0):
    """Mean VN-to-CN message of a degree-i VN (eq. (4), (8), (9)) whose i - 1
    other edges are class d with probability p_frac, class b with q_frac,
    else class a. With p_min > 0: the mean over the VNs with at least p_min
    class-d edges (the weights renormalised)."""
    tot = wsum = 0.0
    a_frac = max(0.0, 1.0 - p_frac - q_frac)
    n = i - 1
    for p in range(p_min, n + 1):
        for q in range(n - p + 1):
            w = (math.comb(n, p) * math.comb(n - p, q) * p_frac ** p * q_frac ** q * a_frac ** (n - p - q))
            if w:
                tot += w * (mu0 + p * mu_d + q * mu_b + (n - p - q) * mu_a)
                wsum += w
    if p_min == 0:
        return tot
    return tot / wsum if wsum > 0 else mu0 + n * mu_a


def _weighted(w, mu):
    """w * mu with a zero weight giving 0 also for an infinite mean."""
    return w * mu if w else 0.0


def _class_d_mean(c_means, b_means, r):
    """Mean of the class-d messages in a sub-iteration: the groups already
    done in this iteration, group 1 by its class-c mean and each later group
    by its class-b and class-c means in the proportions of eq. (5)."""
    if not c_means:
        return 0.0
    terms = [c_means[0]]
    for b, c in zip(b_means[1:], c_means[1:]):
        terms.append(_weighted(r / (1 - r), b) + _weighted((1 - 2 * r) / (1 - r), c))
    return sum(terms) / len(terms)


def _latest_mean(c_means, b_means, r):
    """Mean over all M CNs of each CN's latest message after an iteration,
    in units of N_G CNs: group 1 keeps c_1 on the 1 - r outside the overlap
    with group 2; a middle group keeps b_g on its overlap r and c_g on the
    1 - 2r of its new CNs outside the next overlap; the last group keeps
    b_G on r and c_G on 1 - r. The weights add up to G - (G - 1) r."""
    G = len(c_means)
    if G == 1:
        return c_means[0]
    num = _weighted(1 - r, c_means[0]) + _weighted(r, b_means[-1]) + _weighted(1 - r, c_means[-1])
    for b, c in zip(b_means[1:-1], c_means[1:-1]):
        num += _weighted(r, b) + _weighted(1 - 2 * r, c)
    return num / (G - (G - 1) * r)


def ga_group(dv: int, dc: int, rate: float, ebn0_db: float, G: int, r: float = 0.0, pe: float = 1e-6,
             max_iter: int = 100000):
    """Iterations of the group-shuffled GA recursion (G groups, overlap
    ratio 0 <= r < 0.5; r = 0 is GSBP) until the bit error probability
    drops below pe."""
    if not 0.0 <= r < 0.5:
        raise ValueError("the recursion is implemented for overlap ratios 0 <= r < 0.5")
    lam, rho = _regular(dv, dc)
    mu0 = channel_mean(ebn0_db, rate)
    den = G - (G - 1) * r
    z = r / den if G > 1 else 0.0
    mu_prev = 0.0  # class a: the mean CN message after the previous iteration
    for l in range(1, max_iter + 1):
        cs, bs = [], []  # class-c and class-b CN means of the groups done so far
        for g in range(1, G + 1):
            y = (g - 1) * (1 - r) / den  # class d: CNs of earlier groups outside the overlap
            q = z if g > 1 else 0.0      # class b: the overlap with group g - 1
            mu_d = _class_d_mean(cs, bs, r)
            mu_b = bs[-1] if bs else 0.0
            c = _cn_mean({i: _mixture(i, y, q, mu_prev, mu_d, mu_b, mu0) for i in lam}, lam, rho)
            if q > 0:
                # the overlap CNs: VNs with at least one class-d edge
                b = _cn_mean({i: _mixture(i, y, q, mu_prev, mu_d, mu_b, mu0, p_min=1) for i in lam}, lam, rho)
            else:
                b = c
            cs.append(c)
            bs.append(b)
        # the iteration's CN mean (eq. (17)): every CN's latest message
        new = _latest_mean(cs, bs, r)
        if bit_error(mu0 + dv * new) < pe:
            return l
        if abs(new - mu_prev) <= 1e-14 * max(1.0, new):
            return None
        mu_prev = new
    return None


def threshold(dv: int, dc: int, rate: float, lo: float = 0.0, hi: float = 4.0, steps: int = 40):
    """Smallest Eb/N0 (dB) at which the flooding recursion reaches
    error-free (bisection)."""
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if ga_bp(dv, dc, rate, mid, pe=1e-6, max_iter=20000) is not None:
            hi = mid
        else:
            lo = mid
    return hi


__all__ = ["phi", "phi_inv", "channel_mean", "ga_bp", "ga_group", "threshold"]
