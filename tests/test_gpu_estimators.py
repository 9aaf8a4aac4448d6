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


def _combine(counts, weights, total, k, n, weighted):
    """VSamp's estimate from per-draw counts, in the documented order: weighted,
    term_i = count_i * (Q / (4 w_i)) summed left to right in blocks of 1,024
    draws, the block sums left to right, over k; uniform, the exact integer
    sum times n / (4 k)."""
    if not weighted:
        return (float(int(counts.sum(dtype=np.uint64))) * float(n)) / (4.0 * float(k))
    t = counts.astype(np.float64) * (float(total) / (4.0 * weights.astype(np.float64)))
    parts = [np.cumsum(t[b:b + 1024])[-1] for b in range(0, k, 1024)]
    return float(np.cumsum(parts)[-1]) / float(k)


def test_vsamp_draws_reproduce_vsamp(graph):
    """The draws alone, with the oracle's per-vertex counts at the drawn ids,
    give bfc_vsamp's ids, counts and estimate exactly (uniform and weighted)."""
    nl, nr, l, r, g = graph
    cl, cr = oracle.per_vertex(nl, nr, l, r)
    cnt_all = np.concatenate([cl, cr])
    rng = np.random.default_rng(5)
    probs = rng.random(nl + nr) ** 2
    probs[rng.random(nl + nr) < 0.1] = 0.0
    for k in (1, 1023, 2500):
        for pr in (None, probs):
            seed = 1000 + k
            ids, w, Q = g.vsamp_draws(k, seed, pr)
            vi, vc, ve = g.vsamp(k, seed, pr)
            assert np.array_equal(ids, vi)
            counts = cnt_all[ids]
            assert np.array_equal(counts, vc)
            if pr is None:
                assert Q == nl + nr and np.all(w == 1)
            est = _combine(counts, w, Q, k, nl + nr, pr is not None)
            assert est == ve, (k, pr is None, est, ve)


def test_sparsifiers_and_vsamp_captured_in_one_hip_graph(graph):
    """ESpar, ClrSpar and weighted VSamp queued without any host
    synchronisation, captured once in a HIP graph and replayed with eager
    work between the replays: every replay equals the oracle."""
    import torch
    nl, nr, l, r, g = graph
    dev = g.device
    rng = np.random.default_rng(21)
    probs = torch.as_tensor(rng.random(nl + nr) ** 2).to(dev)
    k = 1500
    want_e = oracle.espar(nl, nr, l, r, 0.3, 77)
    want_c = oracle.clrspar(nl, nr, l, r, 3, 78)
    want_v = oracle.vsamp(nl, nr, l, r, k, 79, probs.cpu().numpy())
    be, bc, bv = g.spar_buffers(), g.spar_buffers(), g.vsamp_buffers(k)

    def queue():
        g.espar_async(be, 0.3, 77)
        g.clrspar_async(bc, 3, 78)
        g.vsamp_async(bv, 79, probs)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        queue()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    hg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(hg):
        queue()
    for i in range(3):
        for t in (be["out"], bc["out"], bv["cnt"], bv["ids"]):
            t.fill_(-1)
        hg.replay()
        torch.cuda.synchronize()
        assert g.spar_result(be) == want_e, i
        assert g.spar_result(bc) == want_c, i
        ids = bv["ids"].cpu().numpy().view(np.uint32)[:k]
        cnt = bv["cnt"].cpu().numpy().view(np.uint64)[:k]
        assert np.array_equal(ids, want_v[0]) and np.array_equal(cnt, want_v[1]), i
        assert float(bv["est"].item()) == want_v[2], i
        assert g.espar(0.5, 5) == oracle.espar(nl, nr, l, r, 0.5, 5)   # eager work between


def test_invalid_probabilities_give_nan_without_synchronising(api):
    import torch
    l, r = gen.biclique(4, 5)
    g = api.Graph(4, 5, l, r)
    buf = g.vsamp_buffers(10)
    bad = torch.tensor(np.r_[np.ones(8), -1.0], dtype=torch.float64, device=g.device)
    g.vsamp_async(buf, 1, bad)
    torch.cuda.synchronize()
    assert np.isnan(float(buf["est"].item()))
    from paper_1801_00338_amd._lib import BfcError
    with pytest.raises(BfcError, match="PROBS"):
        g.check_probs(bad)
