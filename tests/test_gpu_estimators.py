"""GPU parity of the estimators with the CPU oracle for the same seeds.

The random decisions follow one Philox-4x32-10 definition implemented twice
(oracle and HIP), so kept-edge counts, sparsified butterfly counts, drawn
ids and their local counts must match exactly, and the binary64 estimates,
computed in the same fixed order, bit for bit.
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


@pytest.mark.parametrize("p", [1.0, 0.5, 0.1, 0.013])
def test_espar(graph, p):
    nl, nr, l, r, g = graph
    for seed in (1, 2**40 + 3):
        got = g.espar(p, seed)
        want = oracle.espar(nl, nr, l, r, p, seed)
        assert got == want, (p, seed, got, want)


@pytest.mark.parametrize("N", [1, 2, 3, 8, 32])
def test_clrspar(graph, N):
    nl, nr, l, r, g = graph
    for seed in (5, 77):
        got = g.clrspar(N, seed)
        want = oracle.clrspar(nl, nr, l, r, N, seed)
        assert got == want, (N, seed, got, want)


def test_vsamp_uniform_and_weighted(graph):
    nl, nr, l, r, g = graph
    k = 3000
    for seed in (9, 123456789):
        gi, gc, ge = g.vsamp(k, seed)
        oi, oc, oe = oracle.vsamp(nl, nr, l, r, k, seed)
        assert np.array_equal(gi, oi) and np.array_equal(gc, oc) and ge == oe
    rng = np.random.default_rng(3)
    probs = rng.random(nl + nr) ** 3
    probs[rng.random(nl + nr) < 0.2] = 0.0
    for seed in (4, 2**63 + 1):
        gi, gc, ge = g.vsamp(k, seed, probs)
        oi, oc, oe = oracle.vsamp(nl, nr, l, r, k, seed, probs)
        assert np.array_equal(gi, oi) and np.array_equal(gc, oc) and ge == oe


def test_esamp_uniform_and_weighted(graph):
    nl, nr, l, r, g = graph
    k = 2000
    gi, gc, ge = g.esamp(k, 31)
    oi, oc, oe = oracle.esamp(nl, nr, l, r, k, 31)
    assert np.array_equal(gi, oi) and np.array_equal(gc, oc) and ge == oe
    probs = np.random.default_rng(8).random(l.size)
    gi, gc, ge = g.esamp(k, 32, probs)
    oi, oc, oe = oracle.esamp(nl, nr, l, r, k, 32, probs)
    assert np.array_equal(gi, oi) and np.array_equal(gc, oc) and ge == oe


def test_estimator_errors(api):
    from paper_1801_00338_amd._lib import BfcError
    l, r = gen.biclique(4, 5)
    g = api.Graph(4, 5, l, r)
    for bad in (0.0, -0.5, 1.5, float("nan")):
        with pytest.raises(BfcError, match="ARG"):
            g.espar(bad, 1)
    with pytest.raises(BfcError, match="ARG"):
        g.clrspar(0, 1)
    with pytest.raises(BfcError, match="ARG"):
        g.vsamp(0, 1)
    for probs in (np.zeros(9), np.r_[np.ones(8), -1.0], np.r_[np.ones(8), np.nan],
                  np.r_[np.ones(8), np.inf]):
        with pytest.raises(BfcError, match="PROBS"):
            g.vsamp(10, 1, probs)
    # the biclique: every draw proportional to B_v recovers B exactly
    cl, cr = oracle.per_vertex(4, 5, l, r)
    ids, cnt, est = g.vsamp(50, 2, np.concatenate([cl, cr]).astype(np.float64))
    assert est == 60.0
