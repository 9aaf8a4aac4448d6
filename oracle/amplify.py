"""(eps, delta) estimates from the sparsifiers -- TEST INFRASTRUCTURE ONLY.

Plain Python reference for the amplification of Sec. 6 (Sanei-Mehri,
Sariyuce, Tirthapura, "Butterfly Counting in Bipartite Networks"):

- the sampling thresholds of the ESpar lemma (Sec. 6.1) and the ClrSpar
  lemma (Sec. 6.2).  The lemmas claim a variance of at most B^2 / 8, from
  the variance expansions (which count each pair of butterflies once) and
  the observation's pair bounds (which K_{5,5} already breaks: 600 pairs
  sharing a wedge against B Delta = 500).  Counting ordered pairs, a
  butterfly shares a wedge with at most 4 (Delta - 2) others, one edge with
  at most 4 (Delta - 1)^2 and two same-side vertices with at most Delta^2,
  so P_1w <= 4 B Delta, P_1e <= 4 B Delta^2, P_2v <= B Delta^2; above the
  same thresholds one estimate's variance is then below 3 B^2 / 8 (ESpar)
  and 5 B^2 / 16 (ClrSpar), and c = 3/8 serves both;
- the median of means: the mean of r estimates has variance below
  c B^2 / r, so by Chebyshev's inequality it misses B by more than eps B
  with probability at most c / (r eps^2) <= 1/4 for r = ceil(4 c / eps^2) =
  ceil(3 / (2 eps^2)); the median of g such means misses only if at least
  half of them do, which by Hoeffding's inequality happens with probability
  at most exp(-g / 8) <= delta for g = ceil(8 ln(1 / delta)) (made odd, so
  the median is one of the means).

Replica i of a plan is seeded seed + i.
"""
from __future__ import annotations

import math

import oracle


def threshold(kind: str, B: float, max_deg: int):
    """ESpar: p = min(1, max((24/B)^(1/4), sqrt(24 D / B), 24 D^2 / B)).
    ClrSpar: the largest N with 1/N above max((32/B)^(1/3), sqrt(32 D / B),
    32 D^2 / B), at least 1.  B <= 0 (no butterflies expected) keeps everything."""
    if kind == "espar":
        if B <= 0:
            return 1.0
        b = max((24.0 / B) ** 0.25, math.sqrt(24.0 * max_deg / B), 24.0 * max_deg * max_deg / B)
        return min(1.0, b)
    if kind == "clrspar":
        if B <= 0:
            return 1
        b = max((32.0 / B) ** (1.0 / 3.0), math.sqrt(32.0 * max_deg / B),
                32.0 * max_deg * max_deg / B)
        if b >= 1.0:
            return 1
        n = 1
        while 1.0 / (n + 1) > b:        # largest N with 1/N > b
            n += 1
        return n
    raise ValueError(kind)


def plan(eps: float, delta: float):
    """(groups g, estimates per group r) for an (eps, delta) estimate."""
    if not (0 < eps <= 1) or not (0 < delta < 1):
        raise ValueError("need 0 < eps <= 1 and 0 < delta < 1")
    r = math.ceil(3.0 / (2.0 * eps * eps))
    g = math.ceil(8.0 * math.log(1.0 / delta))
    if g % 2 == 0:
        g += 1
    return g, r


def median_of_means(x, g: int, r: int):
    """Group q holds x[q r .. q r + r); its mean sums left to right and divides
    by r; the result is the lower median of the g means."""
    means = []
    for q in range(g):
        s = 0.0
        for i in range(r):
            s += float(x[q * r + i])
        means.append(s / r)
    return means, sorted(means)[(g - 1) // 2]


def spar_eps_delta(nl, nr, l, r, kind, eps, delta, seed, B_pilot, max_deg):
    """The whole estimate: threshold, plan, g r replicas, median of means."""
    param = threshold(kind, B_pilot, max_deg)
    g, rr = plan(eps, delta)
    fn = oracle.espar if kind == "espar" else oracle.clrspar
    est = [fn(nl, nr, l, r, param, seed + i)[1] for i in range(g * rr)]
    means, med = median_of_means(est, g, rr)
    return med, means, param, g, rr
