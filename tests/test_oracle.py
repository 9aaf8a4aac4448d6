"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here touches a GPU.  Each test checks the oracle against something
other than itself: brute-force enumeration of the definitions, closed forms
for complete bipartite graphs, the dataset-table biclique row, identities of
Lemma 1 and Lemma 2, Philox known answers, and estimator special cases.
"""
import json
import os
from itertools import product

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1801_00338_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_graph(rng, nl, nr, m):
    m = min(m, nl * nr)
    keys = rng.choice(nl * nr, size=m, replace=False)
    return (keys // nr).astype(np.uint32), (keys % nr).astype(np.uint32)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ---------------------------------------------------------------- RNG
def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = [int(x, 16) for x in v["out"]]
        assert list(map(int, oracle.philox(ctr, key))) == out


def test_uniform_below_in_range_and_spread():
    n = 7
    xs = [oracle.uniform_below(5, i, 0, oracle.TAG_VDRAW, n) for i in range(7000)]
    assert min(xs) >= 0 and max(xs) < n
    counts = np.bincount(xs, minlength=n)
    chi2 = ((counts - 1000.0) ** 2 / 1000.0).sum()
    assert chi2 < 30.0   # 6 dof; p ~ 4e-5


def test_colors_uniform():
    N = 8
    cs = [oracle.color(11, 1, v, N) for v in range(8000)]
    counts = np.bincount(cs, minlength=N)
    chi2 = ((counts - 1000.0) ** 2 / 1000.0).sum()
    assert chi2 < 35.0


# ---------------------------------------------------------------- exact count
def test_brute_force_two_ways_agree():
    rng = np.random.default_rng(0)
    for _ in range(20):
        nl, nr = rng.integers(1, 7, size=2)
        l, r = rand_graph(rng, nl, nr, rng.integers(0, nl * nr + 1))
        assert brute.butterflies_quadruples(nl, nr, l, r) == len(brute.butterflies(nl, nr, l, r))


def test_exact_vs_brute_random():
    rng = np.random.default_rng(1)
    for _ in range(150):
        nl, nr = rng.integers(1, 13, size=2)
        l, r = rand_graph(rng, nl, nr, rng.integers(0, nl * nr + 1))
        want = brute.butterflies_quadruples(nl, nr, l, r)
        for side in (0, 1, 2):
            assert oracle.exact(nl, nr, l, r, side)[0] == want


def test_exact_all_graphs_3x3():
    cells = [(a, x) for a in range(3) for x in range(3)]
    for mask in range(1 << 9):
        es = [cells[i] for i in range(9) if mask >> i & 1]
        l = np.array([e[0] for e in es], np.uint32)
        r = np.array([e[1] for e in es], np.uint32)
        want = brute.butterflies_quadruples(3, 3, l, r)
        assert oracle.exact(3, 3, l, r)[0] == want


@pytest.mark.parametrize("a,b", [(1, 1), (2, 2), (2, 3), (3, 5), (7, 4), (12, 9), (40, 3)])
def test_complete_bipartite_closed_forms(a, b):
    l, r = gen.biclique(a, b)
    c2 = lambda n: n * (n - 1) // 2
    assert oracle.exact(a, b, l, r)[0] == c2(a) * c2(b)
    cl, cr = oracle.per_vertex(a, b, l, r)
    assert all(int(x) == (a - 1) * c2(b) for x in cl)
    assert all(int(x) == (b - 1) * c2(a) for x in cr)
    ce = oracle.per_edge(a, b, l, r)
    assert all(int(x) == (a - 1) * (b - 1) for x in ce)


def test_dataset_table_biclique_row():
    with open(os.path.join(GOLDEN, "biclique_table2.json")) as f:
        g = json.load(f)
    l, r = gen.biclique(g["n_left"], g["n_right"])
    assert l.size == g["n_edges"]
    sl, sr, _, _ = oracle.degree_stats(g["n_left"], g["n_right"], l, r)
    assert (sl, sr) == (g["sumsq_left"], g["sumsq_right"])
    total, wedges, side = oracle.exact(g["n_left"], g["n_right"], l, r)
    assert total == g["butterflies"]
    # sum_L d^2 < sum_R d^2, so the count starts from R; the work is the
    # number of wedges with midpoint in L (Lemma 2): |L| * C(10, 2).
    assert side == 2 and wedges == g["n_left"] * 45


@pytest.mark.parametrize("k", [3, 4, 5, 8])
def test_even_cycles_and_trees(k):
    # C_{2k}: L_i ~ R_i, R_{i+1}; butterflies only for k = 2.
    l = np.array([i for i in range(k) for _ in range(2)], np.uint32)
    r = np.array([x for i in range(k) for x in (i, (i + 1) % k)], np.uint32)
    assert oracle.exact(k, k, l, r)[0] == 0
    # star, matching, path
    assert oracle.exact(1, k, np.zeros(k, np.uint32), np.arange(k, dtype=np.uint32))[0] == 0
    ar = np.arange(k, dtype=np.uint32)
    assert oracle.exact(k, k, ar, ar)[0] == 0


def test_four_cycle_is_one_butterfly():
    l = np.array([0, 0, 1, 1], np.uint32)
    r = np.array([0, 1, 0, 1], np.uint32)
    assert oracle.exact(2, 2, l, r)[0] == 1


def test_disjoint_union_adds():
    rng = np.random.default_rng(2)
    parts = []
    want = 0
    for _ in range(4):
        nl, nr = rng.integers(2, 20, size=2)
        l, r = rand_graph(rng, nl, nr, rng.integers(0, nl * nr // 2 + 1))
        want += oracle.exact(nl, nr, l, r)[0]
        parts.append((nl, nr, l, r))
    nl, nr, l, r = gen.disjoint_union(parts)
    assert oracle.exact(nl, nr, l, r)[0] == want


def test_invariants_random():
    rng = np.random.default_rng(3)
    for _ in range(25):
        nl, nr = rng.integers(2, 40, size=2)
        l, r = rand_graph(rng, nl, nr, rng.integers(0, nl * nr // 2 + 2))
        B, W, side = oracle.exact(nl, nr, l, r)
        # Eq. (3) and Eq. (4): either side gives the same count
        assert oracle.exact(nl, nr, l, r, 1)[0] == B == oracle.exact(nl, nr, l, r, 2)[0]
        # Lemma 1 (1): per-vertex counts sum to 2B on each side
        cl, cr = oracle.per_vertex(nl, nr, l, r)
        assert int(cl.sum()) == 2 * B == int(cr.sum())
        # every butterfly has four edges
        ce = oracle.per_edge(nl, nr, l, r)
        assert int(ce.sum()) == 4 * B
        # each butterfly through v uses two edges of v
        sl = np.zeros(nl, np.uint64)
        sr = np.zeros(nr, np.uint64)
        np.add.at(sl, l, ce)
        np.add.at(sr, r, ce)
        assert np.array_equal(sl, 2 * cl) and np.array_equal(sr, 2 * cr)
        # relabelling ids and swapping the sides change nothing
        pl, pr = rng.permutation(nl).astype(np.uint32), rng.permutation(nr).astype(np.uint32)
        assert oracle.exact(nl, nr, pl[l], pr[r])[0] == B
        assert oracle.exact(nr, nl, r, l)[0] == B
        # Lemma 2: wedges visited = sum over midpoints of C(d, 2)
        mids = r if side == 1 else l
        d = np.bincount(mids, minlength=nr if side == 1 else nl).astype(np.int64)
        assert W == int((d * (d - 1) // 2).sum())


def test_exact_range_per_start_vs_brute():
    """orc_exact_range: the partial sums of Eq. (3)/(4) over a start range.

    For one start v of the start side, the range [v, v + 1) must give
    sum_{w < v} C(|N(v) & N(w)|, 2) (set intersections written out here) and
    visit sum_{u in N(v)} #{w in N(u): w < v} wedges; disjoint ranges add up
    to the full count, and the full range is orc_exact.
    """
    from math import comb
    rng = np.random.default_rng(8)
    for _ in range(12):
        nl, nr = (int(x) for x in rng.integers(2, 25, size=2))
        l, r = rand_graph(rng, nl, nr, rng.integers(0, nl * nr // 2 + 2))
        B, W, _ = oracle.exact(nl, nr, l, r)
        for side in (1, 2):
            A, Bs, nA = (l, r, nl) if side == 1 else (r, l, nr)
            N = [set() for _ in range(nA)]
            M = {}
            for a, b in zip(A.tolist(), Bs.tolist()):
                N[a].add(b)
                M.setdefault(b, set()).add(a)
            tot = wed = 0
            for v in range(nA):
                want = sum(comb(len(N[v] & N[w]), 2) for w in range(v))
                want_w = sum(sum(1 for w in M[u] if w < v) for u in N[v])
                got, gw, su = oracle.exact_range(nl, nr, l, r, side, v, v + 1)
                assert (got, gw, su) == (want, want_w, side)
                tot += got
                wed += gw
            assert tot == B
            cut = sorted(rng.integers(0, nA + 1, size=2).tolist())
            parts = [oracle.exact_range(nl, nr, l, r, side, a, b)
                     for a, b in ((0, cut[0]), (cut[0], cut[1]), (cut[1], nA))]
            assert sum(p[0] for p in parts) == B
            assert sum(p[1] for p in parts) == oracle.exact(nl, nr, l, r, side)[1]
            assert oracle.exact_range(nl, nr, l, r, side, 0, nA)[:2] == \
                oracle.exact(nl, nr, l, r, side)[:2]
            # an empty or out-of-range slice counts nothing
            assert oracle.exact_range(nl, nr, l, r, side, nA, nA + 5)[:2] == (0, 0)


def test_threads_do_not_change_results():
    """Threads over starts only split the start loop: identical integers."""
    nl, nr = 3_000, 15_000
    l, r = gen.chung_lu(nl, nr, 150_000, 2.1, 2.3, 2000, seed=7)
    try:
        one = (oracle.exact(nl, nr, l, r), oracle.exact_range(nl, nr, l, r, 0, 100, 2_500),
               oracle.per_vertex(nl, nr, l, r), oracle.per_edge(nl, nr, l, r))
        assert oracle.set_threads(4) == 4
        many = (oracle.exact(nl, nr, l, r), oracle.exact_range(nl, nr, l, r, 0, 100, 2_500),
                oracle.per_vertex(nl, nr, l, r), oracle.per_edge(nl, nr, l, r))
    finally:
        oracle.set_threads(1)
    assert one[0] == many[0] and one[1] == many[1]
    assert np.array_equal(one[2][0], many[2][0]) and np.array_equal(one[2][1], many[2][1])
    assert np.array_equal(one[3], many[3])


def test_local_counts_vs_brute():
    rng = np.random.default_rng(4)
    for _ in range(40):
        nl, nr = rng.integers(1, 11, size=2)
        l, r = rand_graph(rng, nl, nr, rng.integers(0, nl * nr + 1))
        bl, br = brute.per_vertex(nl, nr, l, r)
        cl, cr = oracle.per_vertex(nl, nr, l, r)
        assert list(map(int, cl)) == bl and list(map(int, cr)) == br
        be = brute.per_edge(nl, nr, l, r)
        assert list(map(int, oracle.per_edge(nl, nr, l, r))) == be
        for v in range(nl):
            assert oracle.vbfc(nl, nr, l, r, 0, v) == bl[v]
        for v in range(nr):
            assert oracle.vbfc(nl, nr, l, r, 1, v) == br[v]
        for e in range(l.size):
            assert oracle.ebfc(nl, nr, l, r, e) == be[e]


def test_printed_ebfc_fold_overcounts_k23():
    # The fold sum C(C[x], 2) of eBFC as printed gives 3 per edge of K_{2,3};
    # the definition (and the closed form (a-1)(b-1)) gives 2.
    l, r = gen.biclique(2, 3)
    assert brute.per_edge(2, 3, l, r) == [2] * 6
    assert [brute.ebfc_as_printed(2, 3, l, r, e) for e in range(6)] == [3] * 6
    assert list(map(int, oracle.per_edge(2, 3, l, r))) == [2] * 6


def test_errors():
    l = np.array([0, 0], np.uint32)
    r = np.array([1, 1], np.uint32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.exact(1, 2, l, r)
    assert e.value.code == -3
    with pytest.raises(oracle.OracleError) as e:
        oracle.exact(1, 1, l, r)
    assert e.value.code == -2
    with pytest.raises(oracle.OracleError):
        oracle.espar(1, 2, l[:1], r[:1], 0.0, 1)
    with pytest.raises(oracle.OracleError):
        oracle.clrspar(1, 2, l[:1], r[:1], 0, 1)
    with pytest.raises(oracle.OracleError) as e:
        oracle.vsamp(1, 2, l[:1], r[:1], 3, 1, probs=np.array([0.0, -1.0, 1.0]))
    assert e.value.code == -5
    with pytest.raises(oracle.OracleError):
        oracle.vsamp(1, 2, l[:1], r[:1], 3, 1, probs=np.zeros(3))


# ---------------------------------------------------------------- estimators
def _small_dense(seed=5, nl=14, nr=14, m=90):
    rng = np.random.default_rng(seed)
    return (nl, nr) + rand_graph(rng, nl, nr, m)


def test_espar_p1_and_clrspar_n1_are_exact():
    nl, nr, l, r = _small_dense()
    B = oracle.exact(nl, nr, l, r)[0]
    b, est, kept = oracle.espar(nl, nr, l, r, 1.0, 123)
    assert b == B and est == float(B) and kept == l.size
    b, est, kept = oracle.clrspar(nl, nr, l, r, 1, 123)
    assert b == B and est == float(B) and kept == l.size


def test_espar_kept_set_is_subset_and_rate():
    nl, nr, l, r = gen_er = (300, 300) + gen.er(300, 300, 20000, 9)
    kept = [oracle.espar(nl, nr, l, r, 0.25, s)[2] for s in range(20)]
    mean = np.mean(kept) / l.size
    assert abs(mean - 0.25) < 4 * np.sqrt(0.25 * 0.75 / (l.size * 20))


def _variances(nl, nr, l, r):
    B = oracle.exact(nl, nr, l, r)[0]
    t = brute.pair_types(nl, nr, l, r)
    return B, t


def test_sparsifier_means_match_count():
    nl, nr, l, r = _small_dense(6, 16, 16, 110)
    B, t = _variances(nl, nr, l, r)
    assert B > 20
    R = 600
    p = 0.5
    ys = np.array([oracle.espar(nl, nr, l, r, p, s)[1] for s in range(R)])
    var = p ** -8 * (B * (p ** 4 - p ** 8) + 2 * t["1e"] * (p ** 7 - p ** 8)
                     + 2 * t["1w"] * (p ** 6 - p ** 8))
    assert abs(ys.mean() - B) < 4.5 * np.sqrt(var / R)
    N = 2
    q = 1.0 / N
    ys = np.array([oracle.clrspar(nl, nr, l, r, N, s)[1] for s in range(R)])
    var = q ** -6 * (B * (q ** 3 - q ** 6) + 2 * (t["2v"] + t["1e"]) * (q ** 5 - q ** 6)
                     + 2 * t["1w"] * (q ** 4 - q ** 6))
    assert abs(ys.mean() - B) < 4.5 * np.sqrt(var / R)


def test_espar_variance_closed_form_exact_enumeration():
    # Exact E and Var of ESpar by enumerating every kept-edge subset of a
    # small graph, against Lemma 8's expansion with ordered pairs counted.
    nl, nr = 4, 4
    l, r = gen.biclique(3, 4)
    l = np.concatenate([l, np.array([3, 3], np.uint32)])
    r = np.concatenate([r, np.array([0, 1], np.uint32)])
    m = l.size
    idx = {(int(a), int(x)): i for i, (a, x) in enumerate(zip(l, r))}
    masks = []
    for a, b, x, y in brute.butterflies(nl, nr, l, r):
        masks.append(sum(1 << idx[e] for e in ((a, x), (a, y), (b, x), (b, y))))
    B = len(masks)
    t = brute.pair_types(nl, nr, l, r)
    p = 0.3
    ey = ey2 = 0.0
    for s in range(1 << m):
        k = bin(s).count("1")
        w = p ** k * (1 - p) ** (m - k)
        beta = sum(1 for mk in masks if s & mk == mk)
        y = beta / p ** 4
        ey += w * y
        ey2 += w * y * y
    var = ey2 - ey * ey
    closed = p ** -8 * (B * (p ** 4 - p ** 8) + 2 * t["1e"] * (p ** 7 - p ** 8)
                        + 2 * t["1w"] * (p ** 6 - p ** 8))
    assert abs(ey - B) < 1e-9 * B
    assert abs(var - closed) < 1e-7 * closed


def test_clrspar_variance_closed_form_exact_enumeration():
    nl, nr, l, r = _small_dense(8, 3, 4, 9)
    vs = [("L", a) for a in range(nl)] + [("R", x) for x in range(nr)]
    bf = brute.butterflies(nl, nr, l, r)
    B = len(bf)
    assert B > 0
    t = brute.pair_types(nl, nr, l, r)
    N = 2
    ey = ey2 = 0.0
    for cols in product(range(N), repeat=len(vs)):
        c = dict(zip(vs, cols))
        beta = sum(1 for a, b, x, y in bf
                   if c[("L", a)] == c[("L", b)] == c[("R", x)] == c[("R", y)])
        y = beta * N ** 3
        ey += y / N ** len(vs)
        ey2 += y * y / N ** len(vs)
    q = 1.0 / N
    closed = q ** -6 * (B * (q ** 3 - q ** 6) + 2 * (t["2v"] + t["1e"]) * (q ** 5 - q ** 6)
                        + 2 * t["1w"] * (q ** 4 - q ** 6))
    assert abs(ey - B) < 1e-9 * B
    assert abs((ey2 - ey * ey) - closed) < 1e-7 * max(closed, 1)


def test_vsamp_uniform_and_proportional():
    nl, nr, l, r = _small_dense(9, 12, 15, 80)
    B = oracle.exact(nl, nr, l, r)[0]
    cl, cr = oracle.per_vertex(nl, nr, l, r)
    allc = np.concatenate([cl, cr]).astype(np.int64)
    n = nl + nr
    ids, cnt, est = oracle.vsamp(nl, nr, l, r, 4000, 17)
    assert np.array_equal(cnt.astype(np.int64), allc[ids])
    assert est == (float(cnt.sum()) * n) / (4.0 * 4000)
    var1 = n / 16.0 * float((allc ** 2).sum()) - B * B
    assert abs(est - B) < 4.5 * np.sqrt(var1 / 4000)
    # proposal proportional to the local counts: every draw lands on a vertex
    # with B_v > 0 and its Hansen-Hurwitz term is B up to weight quantisation
    ids, cnt, est = oracle.vsamp(nl, nr, l, r, 500, 3, probs=allc.astype(np.float64))
    assert (cnt > 0).all()
    assert abs(est - B) < 1e-6 * B


def test_esamp_uniform():
    nl, nr, l, r = _small_dense(10, 12, 12, 70)
    B = oracle.exact(nl, nr, l, r)[0]
    ce = oracle.per_edge(nl, nr, l, r).astype(np.int64)
    eids, cnt, est = oracle.esamp(nl, nr, l, r, 5000, 21)
    assert np.array_equal(cnt.astype(np.int64), ce[eids.astype(np.int64)])
    var1 = l.size / 16.0 * float((ce ** 2).sum()) - B * B
    assert abs(est - B) < 4.5 * np.sqrt(var1 / 5000)
    eids, cnt, est = oracle.esamp(nl, nr, l, r, 300, 4, probs=ce.astype(np.float64))
    assert abs(est - B) < 1e-6 * B
