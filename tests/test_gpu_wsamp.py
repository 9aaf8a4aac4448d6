"""GPU parity of WSamp (Sec. 5.3) with the CPU oracle for the same seeds.

Wedge numbers come from one Philox-4x32-10 definition on both sides and the
numbering of wedges is fixed, so midpoints, endpoints and counts must match
exactly and the binary64 estimate (an exact integer sum, scaled) bit for bit.
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
    return all(np.array_equal(a, b) for a, b in zip(got[:3], want[:3])) and got[3] == want[3]


@pytest.mark.parametrize("k,seed", [(1, 0), (1000, 5), (5001, 2**40 + 3)])
def test_matches_oracle(graph, k, seed):
    nl, nr, l, r, g = graph
    print(f"k={k} seed={seed}", flush=True)
    assert _same(g.wsamp(k, seed), oracle.wsamp(nl, nr, l, r, k, seed))


def test_special_graphs(api):
    cases = [(4, 5) + gen.biclique(4, 5),
             (1, 6, np.zeros(6, np.uint32), np.arange(6, dtype=np.uint32)),   # star
             (300, 3) + gen.biclique(300, 3),                                 # hubs of 300
             (6, 6, np.array([0, 0, 1, 1, 2], np.uint32), np.array([0, 1, 0, 1, 5], np.uint32))]
    for nl, nr, l, r in cases:
        g = api.Graph(nl, nr, l, r)
        got = g.wsamp(700, 9)
        assert _same(got, oracle.wsamp(nl, nr, l, r, 700, 9))


def test_errors(api):
    from paper_1801_00338_amd._lib import BfcError
    l = np.arange(4, dtype=np.uint32)
    g = api.Graph(4, 4, l, l)                 # a matching: no wedge
    with pytest.raises(BfcError, match="ARG"):
        g.wsamp(10, 1)
    l, r = gen.biclique(3, 3)
    with pytest.raises(BfcError, match="ARG"):
        api.Graph(3, 3, l, r).wsamp(0, 1)


def test_full_size_50m(api):
    """The 1M/5M/50M-edge Chung-Lu graph: 3,000 draws equal the oracle's."""
    w = gen.WORKLOADS["chung_lu_1m_5m_50m"]
    l, r = w.edges()
    print(f"generated {w.name}", flush=True)
    g = api.Graph(w.nl, w.nr, l, r)
    got = g.wsamp(3000, 17)
    print(f"gpu done: est {got[3]:.6g}", flush=True)
    assert _same(got, oracle.wsamp(w.nl, w.nr, l, r, 3000, 17))
