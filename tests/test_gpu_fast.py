"""GPU parity of ESamp with Fast-eBFC (Sec. 5.5) with the CPU oracle.

Edge draws and neighbour picks follow one Philox-4x32-10 definition on both
sides, so drawn edges and hit counts must match exactly and the binary64
estimate, computed in the same fixed order, bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_1801_00338_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1801_00338_amd import api as a
    a.lib()
    oracle.build(force=False)
    return a


GRAPHS = {
    "er": lambda: (2_000, 3_000) + gen.WORKLOADS["er_2k_3k_20k"].edges(),
    "cl": lambda: (3_000, 15_000) + gen.chung_lu(3_000, 15_000, 150_000, 2.1, 2.3, 2000, seed=7),
    "windows": lambda: (200_000, 150_000) + gen.chung_lu(200_000, 150_000, 600_000, 2.2, 2.4,
                                                          5000, seed=11),
}


@pytest.fixture(scope="module", params=list(GRAPHS))
def graph(request, api):
    nl, nr, l, r = GRAPHS[request.param]()
    print(f"graph {request.param} nl={nl} nr={nr} m={l.size}", flush=True)
    return nl, nr, l, r, api.Graph(nl, nr, l, r)


def _same(got, want):
    return (np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
            and got[2] == want[2])


# k = 1 and ragged k; alpha below, at and above one wave's 64 trials
@pytest.mark.parametrize("k,alpha", [(1, 1), (1000, 63), (3001, 64), (777, 65), (500, 1000)])
def test_uniform_matches_oracle(graph, k, alpha):
    nl, nr, l, r, g = graph
    print(f"k={k} alpha={alpha}", flush=True)
    got = g.esamp_fast(k, alpha, 41)
    want = oracle.esamp_fast(nl, nr, l, r, k, alpha, 41)
    assert _same(got, want)
    assert np.array_equal(got[0], g.esamp(k, 41)[0])     # ESamp's draws
    assert (got[1] <= alpha).all()


def test_weighted_matches_oracle(graph):
    nl, nr, l, r, g = graph
    probs = np.random.default_rng(9).random(l.size)
    probs[::7] = 0.0
    got = g.esamp_fast(2049, 100, 2**40 + 5, probs)
    want = oracle.esamp_fast(nl, nr, l, r, 2049, 100, 2**40 + 5, probs)
    assert _same(got, want)


def test_special_graphs(api):
    cases = [(4, 5) + gen.biclique(4, 5),
             (1, 6, np.zeros(6, np.uint32), np.arange(6, dtype=np.uint32)),     # star
             (50, 50, np.arange(50, dtype=np.uint32), np.arange(50, dtype=np.uint32)),
             (300, 3) + gen.biclique(300, 3)]
    for nl, nr, l, r in cases:
        g = api.Graph(nl, nr, l, r)
        got = g.esamp_fast(300, 130, 3)
        assert _same(got, oracle.esamp_fast(nl, nr, l, r, 300, 130, 3))
        if oracle.exact(nl, nr, l, r)[0] == 0:
            assert got[1].sum() == 0 and got[2] == 0.0


def test_errors(api):
    from paper_1801_00338_amd._lib import BfcError
    l, r = gen.biclique(3, 3)
    g = api.Graph(3, 3, l, r)
    for k, alpha in ((0, 5), (5, 0)):
        with pytest.raises(BfcError, match="ARG"):
            g.esamp_fast(k, alpha, 1)
    with pytest.raises(BfcError, match="PROBS"):
        g.esamp_fast(4, 4, 1, np.r_[np.ones(8), -1.0])


def test_full_size_50m(api):
    """The 1M/5M/50M-edge Chung-Lu graph: 2,000 draws of 1,000 trials equal the
    oracle's draw for draw."""
    import torch
    w = gen.WORKLOADS["chung_lu_1m_5m_50m"]
    l, r = w.edges()
    print(f"generated {w.name}", flush=True)
    g = api.Graph(w.nl, w.nr, l, r)
    got = g.esamp_fast(2000, 1000, 7)
    torch.cuda.synchronize()
    print(f"gpu done: est {got[2]:.6g}", flush=True)
    want = oracle.esamp_fast(w.nl, w.nr, l, r, 2000, 1000, 7)
    assert _same(got, want)
