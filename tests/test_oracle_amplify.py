"""Pins of the (eps, delta) amplification reference (Sec. 6.1, 6.2).

- The per-butterfly pair bounds that the variance guarantee rests on, by
  brute force (ordered pairs: P_1w <= 4 B D, P_1e <= 4 B D^2, P_2v <= B D^2),
  and the counterexample to the paper's unordered p_1w <= B D on K_{5,5}.
- The plan's sizes meet Chebyshev's and Hoeffding's conditions.
- The median of means on inputs whose answer is known.
- End to end on a graph whose threshold is below 1: the (eps, delta)
  estimate misses by more than eps B in at most a delta share of seeds.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import amplify, brute
from paper_1801_00338_amd import gen


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _rand_graph(seed, nl, nr, m):
    rng = np.random.default_rng(seed)
    keys = rng.choice(nl * nr, size=min(m, nl * nr), replace=False)
    return nl, nr, (keys // nr).astype(np.uint32), (keys % nr).astype(np.uint32)


def _max_deg(nl, nr, l, r):
    return int(max(np.bincount(l, minlength=nl).max(), np.bincount(r, minlength=nr).max()))


@pytest.mark.parametrize("name", ["k55", "k37", "r1", "r2", "r3"])
def test_pair_bounds(name):
    if name == "k55":
        nl, nr, (l, r) = 5, 5, gen.biclique(5, 5)
    elif name == "k37":
        nl, nr, (l, r) = 3, 7, gen.biclique(3, 7)
    else:
        nl, nr, l, r = _rand_graph({"r1": 1, "r2": 2, "r3": 3}[name], 9, 8, 45)
    B = len(brute.butterflies(nl, nr, l, r))
    D = _max_deg(nl, nr, l, r)
    t = brute.pair_types(nl, nr, l, r)          # unordered pairs
    assert 2 * t["1w"] <= 4 * B * (D - 2)
    assert 2 * t["1e"] <= 4 * B * (D - 1) ** 2
    assert 2 * t["2v"] <= B * D * D
    if name == "k55":
        assert t["1w"] == 600 and B * D == 500   # the paper's p_1w <= B D fails


def test_plan_sizes():
    for eps, delta in ((0.01, 0.05), (0.1, 0.01), (0.3, 0.2), (1.0, 0.5)):
        g, r = amplify.plan(eps, delta)
        assert 3 / 8 / (r * eps * eps) <= 0.25          # Chebyshev per group
        assert math.exp(-g / 8) <= delta and g % 2 == 1  # Hoeffding on the median
    for bad in ((0.0, 0.1), (0.1, 0.0), (0.1, 1.0), (1.5, 0.1)):
        with pytest.raises(ValueError):
            amplify.plan(*bad)


def test_thresholds():
    # tiny counts keep everything; the ClrSpar N is the largest with 1/N above the bound
    assert amplify.threshold("espar", 10.0, 5) == 1.0
    assert amplify.threshold("clrspar", 10.0, 5) == 1
    B, D = 1e12, 100
    b = max((32 / B) ** (1 / 3), math.sqrt(32 * D / B), 32 * D * D / B)
    n = amplify.threshold("clrspar", B, D)
    assert 1 / n > b >= 1 / (n + 1)
    p = amplify.threshold("espar", B, D)
    assert p == max((24 / B) ** 0.25, math.sqrt(24 * D / B), 24 * D * D / B) and p < 1


def test_median_of_means_known_answer():
    # group means 3, 1, 2 (each from values summed left to right): median 2
    x = [2.0, 4.0, 1.0, 1.0, 0.5, 3.5]
    means, med = amplify.median_of_means(x, 3, 2)
    assert means == [3.0, 1.0, 2.0] and med == 2.0
    means, med = amplify.median_of_means([5.0, 1.0, 7.0, 7.0, 3.0], 5, 1)
    assert med == 5.0


def test_eps_delta_guarantee_end_to_end():
    nl, nr, l, r = _rand_graph(7, 30, 30, 470)
    B = oracle.exact(nl, nr, l, r)[0]
    D = _max_deg(nl, nr, l, r)
    p = amplify.threshold("espar", B, D)
    assert p < 1.0, (B, D)
    eps, delta, T = 0.3, 0.2, 30
    miss = 0
    for t in range(T):
        med, means, param, g, rr = amplify.spar_eps_delta(nl, nr, l, r, "espar", eps, delta,
                                                          1000 * t, B, D)
        miss += abs(med - B) > eps * B
    assert miss <= delta * T
