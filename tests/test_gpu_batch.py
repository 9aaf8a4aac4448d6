"""GPU parity of batched counting (many graphs, many sparsifier replicas) with the oracle.

Per-graph totals of a batch and per-replica counts and estimates are integer
or fixed-expression binary64 results: they must equal the oracle's (and the
single-graph calls') exactly.
"""
import math
import time

import numpy as np
import pytest

import oracle
from paper_1801_00338_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1801_00338_amd import api
    api.lib()
    oracle.build(force=False)
    return torch, api


def _special_graphs():
    """Edge cases: empty, single vertex sides, a biclique, a hub start, a matching."""
    out = [(5, 7, np.zeros(0, np.uint32), np.zeros(0, np.uint32)),
           (1, 1, np.array([0], np.uint32), np.array([0], np.uint32))]
    l, r = gen.biclique(6, 9)
    out.append((6, 9, l, r))
    l, r = gen.biclique(300, 3)          # R starts of degree 300 (> 255: the wide kernel)
    out.append((300, 3, l, r))
    out.append((50, 50, np.arange(50, dtype=np.uint32), np.arange(50, dtype=np.uint32)))
    nl, nr = 400, 3000
    l, r = gen.chung_lu(nl, nr, 20_000, 2.1, 2.1, 900, seed=17)
    out.append((nl, nr, l, r))
    return out


def _oracle_totals(graphs):
    tot, side = [], []
    for nl, nr, l, r in graphs:
        b, _, s = oracle.exact(nl, nr, l, r)
        tot.append(b)
        side.append(s)
    return np.array(tot, np.uint64), np.array(side)


@pytest.fixture(scope="module")
def small_batch(env):
    torch, api = env
    graphs = gen.batch_graphs(40, 100, 20_000, seed=3) + _special_graphs()
    print(f"small batch: {len(graphs)} graphs, m={sum(len(g[2]) for g in graphs)}", flush=True)
    b = api.Batch(graphs)
    want, side = _oracle_totals(graphs)
    return graphs, b, want, side


def test_batch_totals_match_oracle(small_batch):
    graphs, b, want, side = small_batch
    got = b.totals()
    assert np.array_equal(got, want)
    # each graph entered from the side ExactBFC's rule picks (the oracle's side 2 = R)
    assert np.array_equal(b.swapped, side == 2)
    assert b.wedges == sum(oracle.exact(*g)[1] for g in graphs)


@pytest.mark.parametrize("tuning", [
    dict(narrow_max=255, chunk=1), dict(narrow_max=127, chunk=16), dict(narrow_max=31, chunk=4),
    dict(narrow_max=1, chunk=64), dict(narrow_waves_per_cu=1, wide_groups_per_cu=1),
    dict(narrow_waves_per_cu=5, wide_groups_per_cu=2, narrow_max=200)])
def test_batch_tunings(small_batch, tuning):
    graphs, b, want, _ = small_batch
    print(f"tuning {tuning}", flush=True)
    assert np.array_equal(b.totals(tuning), want)


def test_bad_tuning_rejected(small_batch, env):
    _, api = env
    graphs, b, _, _ = small_batch
    from paper_1801_00338_amd._lib import BfcError
    for t in (dict(narrow_max=256), dict(chunk=65), dict(narrow_waves_per_cu=9),
              dict(wide_groups_per_cu=3)):
        with pytest.raises(BfcError):
            b.totals(t)


def test_autotune_picks_a_valid_shape(small_batch):
    graphs, b, want, _ = small_batch
    best, ms = b.autotune()
    print(f"autotune: {best.as_dict()} {ms:.3f} ms", flush=True)
    assert ms > 0 and 1 <= best.narrow_max <= 255
    assert np.array_equal(b.totals(best), want)


def test_exact_tuned_single_graph(env):
    torch, api = env
    nl, nr = 3_000, 15_000
    l, r = gen.chung_lu(nl, nr, 150_000, 2.1, 2.3, 2000, seed=7)
    g = api.Graph(nl, nr, l, r)
    want = oracle.exact(nl, nr, l, r)[0]
    for t in (None, dict(narrow_max=63, chunk=2), dict(narrow_waves_per_cu=3)):
        assert g.exact_tuned(t) == want
    best, ms = g.autotune()
    assert g.exact_tuned(best) == want


def test_batch_hip_graph_replays(small_batch, env):
    """The batched count captured once in a HIP graph and replayed several times,
    with eager work and synchronisations between replays; every replay must
    equal the eager result."""
    torch, api = env
    graphs, b, want, _ = small_batch
    out = torch.zeros(b.n_graphs, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.totals_async(out, stream=s)          # warm the kernels outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.totals_async(out)
    for i in range(4):
        out.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, want), i
        assert np.array_equal(b.totals(), want)      # eager work between replays


# ------------------------------------------------------------------ replica batches
REPLICAS = ([("espar", p, sd) for p in (1.0, 0.5, 0.1, 0.013) for sd in (1, 2**40 + 3)] +
            [("clrspar", n, sd) for n in (1, 2, 3, 8, 32) for sd in (5, 77)])


def test_spar_batch_matches_single_calls_and_oracle(env):
    torch, api = env
    nl, nr = 3_000, 15_000
    l, r = gen.chung_lu(nl, nr, 150_000, 2.1, 2.3, 2000, seed=7)
    g = api.Graph(nl, nr, l, r)
    beta, est, kept = g.spar_batch(REPLICAS)
    for i, (kind, param, sd) in enumerate(REPLICAS):
        single = g.espar(param, sd) if kind == "espar" else g.clrspar(param, sd)
        want = (oracle.espar if kind == "espar" else oracle.clrspar)(nl, nr, l, r, param, sd)
        assert (int(beta[i]), float(est[i]), int(kept[i])) == want == single, (kind, param, sd)


def test_spar_batch_hip_graph_replays(env):
    """Phase 2 of a replica batch captured once in a HIP graph and replayed
    several times, with eager work between replays: every replay equals the
    eager run and the single-replica calls."""
    torch, api = env
    nl, nr = 3_000, 15_000
    l, r = gen.chung_lu(nl, nr, 150_000, 2.1, 2.3, 2000, seed=7)
    g = api.Graph(nl, nr, l, r)
    rb = api.ReplicaBatch(g, REPLICAS)
    want_b, want_e = rb.run()
    n = len(REPLICAS)
    beta = torch.zeros(n, dtype=torch.int64, device="cuda")
    est = torch.zeros(n, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        rb.run_async(beta, est, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rb.run_async(beta, est)
    for i in range(4):
        beta.fill_(-1)
        est.fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(beta.cpu().numpy().view(np.uint64), want_b), i
        assert np.array_equal(est.cpu().numpy(), want_e), i
        kind, param, sd = REPLICAS[i]
        single = g.espar(param, sd) if kind == "espar" else g.clrspar(param, sd)
        assert (int(want_b[i]), float(want_e[i]), int(rb.kept[i])) == single


def test_spar_batch_rejects_foreign_sizes(env):
    """Phase 2 laid out from another replica set's sizes marks every result
    invalid instead of reading or writing outside its buffers."""
    torch, api = env
    nl, nr = 3_000, 15_000
    l, r = gen.chung_lu(nl, nr, 150_000, 2.1, 2.3, 2000, seed=7)
    g = api.Graph(nl, nr, l, r)
    rb = api.ReplicaBatch(g, [("espar", 0.5, 1), ("clrspar", 4, 2)])
    other = api.ReplicaBatch(g, [("espar", 0.5, 3), ("clrspar", 4, 4)])
    # phase 2 of rb's seeds laid out (and its workspace sized) from other's sizes:
    # the check on the device must fail
    rb.info, rb.ws = other.info, other.ws
    beta, est = rb.run()
    assert np.all(beta == np.uint64(2**64 - 1)) and np.all(np.isnan(est))


def test_spar_batch_edge_cases(env):
    torch, api = env
    from paper_1801_00338_amd._lib import BfcError
    l, r = gen.biclique(4, 5)
    g = api.Graph(4, 5, l, r)
    beta, est, kept = g.spar_batch([("espar", 1.0, 1), ("clrspar", 1, 2), ("espar", 1e-9, 3)])
    B = math.comb(4, 2) * math.comb(5, 2)
    assert list(beta) == [B, B, 0] and list(kept)[:2] == [20, 20] and est[2] == 0.0
    with pytest.raises(BfcError):
        g.spar_batch([("espar", 0.0, 1)])
    with pytest.raises(BfcError):
        g.spar_batch([("clrspar", 0, 1)])


# ------------------------------------------------------------------ full sizes
def test_full_replica_batch_256(env):
    """256 replicas of the 10M/30M/100M-edge graph in one batch: 128 ESpar (32
    each at p = 0.01, 0.02, 0.05, 0.1) and 128 ClrSpar (32 each at N = 4, 8,
    16, 32), replica r seeded (4 << 32) | r.  Sampled replicas equal the
    oracle and the single-replica calls bit for bit; every group's mean
    estimate lies within four standard errors of the exact count."""
    torch, api = env
    w = gen.WORKLOADS["chung_lu_10m_30m_100m"]
    t0 = time.time()
    l, r = w.edges()
    print(f"generated {w.name} in {time.time() - t0:.1f} s", flush=True)
    g = api.Graph(w.nl, w.nr, l, r)
    B = g.exact()
    print(f"graph built and counted: B={B}", flush=True)
    reps = []
    for p in (0.01, 0.02, 0.05, 0.1):
        reps += [("espar", p, (4 << 32) | len(reps) + i) for i in range(32)]
    for n in (4, 8, 16, 32):
        reps += [("clrspar", n, (4 << 32) | len(reps) + i) for i in range(32)]
    t0 = time.time()
    rb = api.ReplicaBatch(g, reps, log=lambda msg: print(msg, flush=True))
    beta, est = rb.run()
    kept = rb.kept
    print(f"B={B}; batch of {len(reps)} replicas, {int(kept.sum())} kept edges, workspace "
          f"{rb.ws_bytes / 1e9:.1f} GB, {time.time() - t0:.1f} s", flush=True)
    for grp in range(8):
        e = est[32 * grp:32 * grp + 32]
        kind, param, _ = reps[32 * grp]
        se = e.std(ddof=1) / math.sqrt(32)
        print(f"{kind} {param}: mean {e.mean():.6g} rel.err {(e.mean() - B) / B:+.4f} "
              f"std {e.std(ddof=1):.4g}", flush=True)
        assert abs(e.mean() - B) <= 4 * se + 1e-9 * B, (kind, param)
    # sampled replicas: the oracle on the cheapest, single GPU calls on others
    for i in (0, 32 * 7 + 5):
        kind, param, sd = reps[i]
        want = (oracle.espar if kind == "espar" else oracle.clrspar)(w.nl, w.nr, l, r, param, sd)
        assert (int(beta[i]), float(est[i]), int(kept[i])) == want, (kind, param, sd)
    for i in (32 * 3 + 1, 32 * 4 + 2):
        kind, param, sd = reps[i]
        single = g.espar(param, sd) if kind == "espar" else g.clrspar(param, sd)
        assert (int(beta[i]), float(est[i]), int(kept[i])) == single, (kind, param, sd)
