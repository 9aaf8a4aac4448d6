"""GPU results at the full workload sizes against the oracle's stored values.

tests/golden/full_size.json is written by tests/golden/make_full_size.py, which
calls only the CPU oracle (ExactBFC, Sec. 4; the local counts of Sec. 4.2 and
Eq. (2)).  Each entry keeps the SHA-256 of its input edge arrays: a mismatch
there means the generator changed (the stored values are then stale), not
that a count is wrong.  Totals are compared as uint64 integers, per-vertex and
per-edge arrays through the SHA-256 of their little-endian uint64 bytes (and
their sums).
"""
import hashlib
import json
import os
import time

import numpy as np
import pytest

from paper_1801_00338_amd import gen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size.json")


def golden(name):
    with open(GOLDEN) as f:
        d = json.load(f)
    if name not in d:
        pytest.fail(f"{name} missing from {GOLDEN}: run tests/golden/make_full_size.py {name}")
    return d[name]


def edge_sha(l, r):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(l, "<u4").tobytes())
    h.update(np.ascontiguousarray(r, "<u4").tobytes())
    return h.hexdigest()


def u64_sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, "<u8").tobytes())
    return h.hexdigest()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1801_00338_amd import api
    api.lib()
    return torch, api


def _graph(api, name):
    want = golden(name)
    w = gen.WORKLOADS[name]
    t = time.time()
    l, r = w.edges()
    print(f"{name}: generated m={l.size} in {time.time() - t:.0f} s", flush=True)
    assert edge_sha(l, r) == want["edges_sha256"], "generator output differs from the golden input"
    g = api.Graph(w.nl, w.nr, l, r)
    return w, g, want


def test_chung_lu_1m_5m_50m_total_and_local_counts(env):
    torch, api = env
    w, g, want = _graph(api, "chung_lu_1m_5m_50m")
    assert g.wedges() == want["wedges"]
    assert g.side_used() == (1 if want["side"] == "L" else 2)
    assert g.exact() == want["total"]
    print("chung_lu_1m_5m_50m: total agrees", flush=True)
    cl, cr, ce = g.local()
    assert int(cl.sum(dtype=np.uint64)) == want["per_vertex_sum_l"]
    assert int(cr.sum(dtype=np.uint64)) == want["per_vertex_sum_r"]
    assert int(ce.sum(dtype=np.uint64)) == want["per_edge_sum"]
    assert u64_sha(cl, cr) == want["per_vertex_sha256"]
    assert u64_sha(ce) == want["per_edge_sha256"]


@pytest.mark.parametrize("name", ["chung_lu_10m_30m_100m", "chung_lu_20m_80m_400m"])
def test_large_graph_totals(env, name):
    torch, api = env
    w, g, want = _graph(api, name)
    assert g.wedges() == want["wedges"]
    assert g.side_used() == (1 if want["side"] == "L" else 2)
    got = g.exact()
    print(f"{name}: B={got}", flush=True)
    assert got == want["total"]


def test_batch_1024_totals_eager_and_captured(env):
    """The 1,024 uneven graphs: every per-graph total equals the oracle's, in
    an eager call and in each replay of the call captured in a HIP graph."""
    torch, api = env
    want = golden("batch_1024")
    spec = want["input"]
    t = time.time()
    graphs = gen.batch_graphs(spec["count"], spec["m_lo"], spec["m_hi"], seed=spec["seed"])
    h = hashlib.sha256()
    for _, _, l, r in graphs:
        h.update(edge_sha(l, r).encode())
    print(f"batch_1024: generated in {time.time() - t:.0f} s", flush=True)
    assert h.hexdigest() == want["edges_sha256"], "generator output differs from the golden input"
    b = api.Batch(graphs)
    del graphs
    expect = np.array(want["totals"], dtype=np.uint64)
    assert np.array_equal(b.swapped, np.array([s == "R" for s in want["sides"]]))
    assert np.array_equal(b.totals(), expect)
    print("batch_1024: eager totals agree", flush=True)
    out = torch.zeros(b.n_graphs, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.totals_async(out, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.totals_async(out)
    for i in range(3):
        out.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint64), expect), i
    print("batch_1024: captured replays agree", flush=True)
