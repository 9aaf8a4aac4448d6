"""Pins of the oracle's ESamp with Fast-eBFC (Sec. 5.5) against the mathematics.

- Lemma of Sec. 5.5: over all d_a * d_x picks of the two neighbours exactly
  B_e pairs close a butterfly.  Checked by exhaustion against brute-force
  per-edge counts, so a wrong hit test (a dropped b != a, a transposed
  probe) fails it.
- The edge draws are ESamp's draws (the same stream).
- Unbiasedness per edge: hits * d_a * d_x / alpha over many trials sits
  within a few standard deviations sqrt(B_e (d_a d_x - B_e) / alpha) of
  B_e, which catches a biased neighbour pick (an index that never reaches
  the last neighbour, a skew in the draw).
- Unbiasedness of the estimate over seeds, against the exact variance of one
  draw, uniform and weighted.
- Graphs without butterflies never hit.
"""
import math

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


def _deg_products(nl, nr, l, r):
    dl = np.bincount(l, minlength=nl).astype(np.int64)
    dr = np.bincount(r, minlength=nr).astype(np.int64)
    return dl[l] * dr[r]


@pytest.mark.parametrize("graph", ["k23", "k45", "rand1", "rand2", "star"])
def test_hitting_pairs_equal_per_edge_count(graph):
    if graph == "k23":
        nl, nr = 2, 3
        l, r = gen.biclique(2, 3)
    elif graph == "k45":
        nl, nr = 4, 5
        l, r = gen.biclique(4, 5)
    elif graph == "star":
        nl, nr = 1, 6
        l, r = np.zeros(6, np.uint32), np.arange(6, dtype=np.uint32)
    else:
        nl, nr, l, r = _rand_graph(3 if graph == "rand1" else 8, 7, 8, 30)
    want = brute.per_edge(nl, nr, l, r)
    got = [oracle.fast_ebfc_pairs(nl, nr, l, r, e) for e in range(l.size)]
    assert got == want


def test_edge_draws_are_esamp_draws():
    nl, nr, l, r = _rand_graph(11, 12, 12, 70)
    for seed in (0, 5, 2**40 + 9):
        e1, _, _ = oracle.esamp(nl, nr, l, r, 300, seed)
        e2, _, _ = oracle.esamp_fast(nl, nr, l, r, 300, 3, seed)
        assert np.array_equal(e1, e2)
    probs = np.random.default_rng(2).random(l.size)
    e1, _, _ = oracle.esamp(nl, nr, l, r, 300, 7, probs=probs)
    e2, _, _ = oracle.esamp_fast(nl, nr, l, r, 300, 3, 7, probs=probs)
    assert np.array_equal(e1, e2)


def test_trials_unbiased_per_edge():
    nl, nr, l, r = _rand_graph(4, 9, 10, 45)
    ce = np.array(brute.per_edge(nl, nr, l, r), np.float64)
    dd = _deg_products(nl, nr, l, r).astype(np.float64)
    alpha = 100_000
    eids, hits, _ = oracle.esamp_fast(nl, nr, l, r, 40, alpha, 123)
    eids = eids.astype(np.int64)
    z = hits.astype(np.float64) * dd[eids] / alpha
    b = ce[eids]
    sd = np.sqrt(b * (dd[eids] - b) / alpha)
    assert np.all(hits[b == 0] == 0)
    assert np.all(np.abs(z - b) <= 5 * sd + 1e-12)
    assert (b > 0).sum() >= 20


def _single_draw_variance(ce, dd, alpha, w=None):
    """Variance of one draw's term: the edge draw plus the trials' binomial part."""
    ez2 = ce * ce + ce * (dd - ce) / alpha          # E[Z_e^2] of the per-edge estimate
    B = ce.sum() / 4
    if w is None:
        m = ce.size
        return (m / 4) ** 2 * ez2.mean() - B * B
    q = w / w.sum()
    return float((ez2 / (16 * q))[q > 0].sum()) - B * B


def test_estimate_mean_and_variance_uniform():
    nl, nr, l, r = _rand_graph(6, 10, 11, 60)
    ce = np.array(brute.per_edge(nl, nr, l, r), np.float64)
    dd = _deg_products(nl, nr, l, r).astype(np.float64)
    B = ce.sum() / 4
    k, alpha, T = 100, 8, 300
    ests = np.array([oracle.esamp_fast(nl, nr, l, r, k, alpha, (5 << 40) | t)[2]
                     for t in range(T)])
    v1 = _single_draw_variance(ce, dd, alpha)
    assert abs(ests.mean() - B) <= 4.5 * math.sqrt(v1 / (k * T))
    # the spread of the estimate matches the variance of k draws
    assert 0.7 < ests.var(ddof=1) / (v1 / k) < 1.4


def test_estimate_mean_weighted():
    nl, nr, l, r = _rand_graph(6, 10, 11, 60)
    ce = np.array(brute.per_edge(nl, nr, l, r), np.float64)
    dd = _deg_products(nl, nr, l, r).astype(np.float64)
    B = ce.sum() / 4
    probs = ce + 0.5 * ce.mean()
    q = np.maximum(1, np.floor(probs / probs.max() * (2**32 - 1)))
    k, alpha, T = 100, 8, 300
    ests = np.array([oracle.esamp_fast(nl, nr, l, r, k, alpha, t, probs=probs)[2]
                     for t in range(T)])
    v1 = _single_draw_variance(ce, dd, alpha, q)
    assert abs(ests.mean() - B) <= 4.5 * math.sqrt(v1 / (k * T))


def test_no_butterflies_never_hit():
    # a path and a matching plus a star: no 4-cycle anywhere
    l = np.array([0, 0, 1, 1, 2, 3, 4, 4, 4], np.uint32)
    r = np.array([0, 1, 1, 2, 3, 4, 5, 6, 7], np.uint32)
    assert oracle.exact(5, 8, l, r)[0] == 0
    eids, hits, est = oracle.esamp_fast(5, 8, l, r, 50, 64, 1)
    assert hits.sum() == 0 and est == 0.0


def test_errors():
    l, r = gen.biclique(2, 2)
    for args in ((0, 4, 1), (4, 0, 1), (2**32, 4, 1)):
        with pytest.raises(oracle.OracleError):
            oracle.esamp_fast(2, 2, l, r, *args)
    with pytest.raises(oracle.OracleError):
        oracle.fast_ebfc_pairs(2, 2, l, r, 4)
