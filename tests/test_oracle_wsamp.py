"""Pins of the oracle's WSamp (Sec. 5.3) against the mathematics.

- Decoding every wedge number 0 .. W-1 lists every wedge of the graph exactly
  once (compared with a brute-force enumeration over neighbour pairs), so a
  uniform number is a uniform wedge (the lemma of Sec. 5.3).
- Each wedge's count equals the brute-force number of butterflies through it,
  and the counts over all wedges sum to 4B (each butterfly has four wedges),
  so the estimate is unbiased.
- The sampler's draws are the decoded numbers of the pinned uniform stream.
- The mean over seeds matches B within the exact variance of one draw.
"""
import math
from itertools import combinations

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1801_00338_amd import gen


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _rand_graph(seed, nl, nr, m):
    rng = np.random.default_rng(seed)
    keys = rng.choice(nl * nr, size=min(m, nl * nr), replace=False)
    return nl, nr, (keys // nr).astype(np.uint32), (keys % nr).astype(np.uint32)


def _brute_wedges(nl, nr, l, r):
    """{(midpoint, frozenset(ends)): butterflies through it}, global ids."""
    nb = {}
    for a, x in zip(l.tolist(), r.tolist()):
        nb.setdefault(a, set()).add(nl + x)
        nb.setdefault(nl + x, set()).add(a)
    out = {}
    for u, ns in nb.items():
        for v, w in combinations(sorted(ns), 2):
            out[(u, frozenset((v, w)))] = len(nb[v] & nb[w]) - 1
    return out


GRAPHS = {
    "k23": lambda: (2, 3) + gen.biclique(2, 3),
    "k45": lambda: (4, 5) + gen.biclique(4, 5),
    "rand1": lambda: _rand_graph(1, 7, 9, 30),
    "rand2": lambda: _rand_graph(2, 12, 6, 40),
    "isolated": lambda: (6, 6, np.array([0, 0, 1, 1, 2], np.uint32),
                         np.array([0, 1, 0, 1, 5], np.uint32)),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_every_wedge_once_with_its_count(name):
    nl, nr, l, r = GRAPHS[name]()
    mids, ends, cnt, W = oracle.wedges(nl, nr, l, r)
    want = _brute_wedges(nl, nr, l, r)
    got = {}
    for u, (v, w), c in zip(mids.tolist(), ends.tolist(), cnt.tolist()):
        assert v != w
        key = (u, frozenset((v, w)))
        assert key not in got
        got[key] = c
    assert W == len(want) and got == want
    B = len(brute.butterflies(nl, nr, l, r))
    assert int(cnt.sum()) == 4 * B


def test_pair_numbering_inside_a_midpoint():
    # a star of degree 5 in L: numbers run over the pairs (0,1), (0,2), (1,2), (0,3), ...
    l = np.zeros(5, np.uint32)
    r = np.arange(5, dtype=np.uint32)
    mids, ends, _, W = oracle.wedges(1, 5, l, r)
    assert W == 10 and (mids == 0).all()
    # all R degrees are 1, so the neighbour order is the id order
    pairs = [(int(a) - 1, int(b) - 1) for a, b in ends]
    assert pairs == [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (2, 3), (0, 4), (1, 4), (2, 4),
                     (3, 4)]


def test_draws_are_decoded_uniform_numbers():
    nl, nr, l, r = _rand_graph(3, 10, 11, 50)
    _, _, _, W = oracle.wedges(nl, nr, l, r)
    k, seed = 200, 2**33 + 1
    mids, ends, cnt, est = oracle.wsamp(nl, nr, l, r, k, seed)
    t = [oracle.uniform_below(seed, i, 0, oracle.TAG_WDRAW, W) for i in range(k)]
    m2, e2, c2, _ = oracle.wedges(nl, nr, l, r, t)
    assert np.array_equal(mids, m2) and np.array_equal(ends, e2) and np.array_equal(cnt, c2)
    assert est == (float(cnt.sum()) * W) / (4.0 * k)


def test_estimate_mean_over_seeds():
    nl, nr, l, r = _rand_graph(5, 10, 11, 60)
    _, _, cnt, W = oracle.wedges(nl, nr, l, r)
    c = cnt.astype(np.float64)
    B = c.sum() / 4
    v1 = (W / 4) ** 2 * float(np.mean(c * c)) - B * B
    k, T = 100, 400
    ests = np.array([oracle.wsamp(nl, nr, l, r, k, (5 << 40) | s)[3] for s in range(T)])
    assert abs(ests.mean() - B) <= 4.5 * math.sqrt(v1 / (k * T))
    assert 0.75 < ests.var(ddof=1) / (v1 / k) < 1.3


def test_errors():
    # no vertex of degree 2: no wedge to draw
    l = np.arange(4, dtype=np.uint32)
    with pytest.raises(oracle.OracleError):
        oracle.wsamp(4, 4, l, l, 10, 1)
    l, r = gen.biclique(2, 2)
    with pytest.raises(oracle.OracleError):
        oracle.wsamp(2, 2, l, r, 0, 1)
    with pytest.raises(oracle.OracleError):
        oracle.wedges(2, 2, l, r, [4])
