"""GPU parity: the HIP library against the CPU oracle, element by element.

Every call goes through the C ABI (paper_1801_00338_amd.api -> libbfc.so).
Exact counts are integers and must match bit for bit.
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


def rand_graph(rng, nl, nr, m):
    m = min(m, nl * nr)
    keys = rng.choice(nl * nr, size=m, replace=False)
    return (keys // nr).astype(np.uint32), (keys % nr).astype(np.uint32)


def check_all(api, nl, nr, l, r, local=True, sides=(0, 1, 2)):
    print(f"case nl={nl} nr={nr} m={l.size}", flush=True)
    g = api.Graph(nl, nr, l, r)
    want = oracle.exact(nl, nr, l, r)[0]
    for side in sides:
        got = g.exact(side)
        assert got == want, (side, got, want)
    sl, sr, ml, mr = oracle.degree_stats(nl, nr, l, r)
    assert g.sumsq == (sl, sr)
    assert g.max_degree == (ml, mr)
    if local:
        cl, cr, ce = g.local()
        ol, orr = oracle.per_vertex(nl, nr, l, r)
        oe = oracle.per_edge(nl, nr, l, r)
        assert np.array_equal(cl, ol)
        assert np.array_equal(cr, orr)
        assert np.array_equal(ce, oe)
    return want


def test_tiny_random_graphs(api):
    rng = np.random.default_rng(100)
    for _ in range(60):
        nl, nr = rng.integers(1, 30, size=2)
        l, r = rand_graph(rng, nl, nr, rng.integers(0, nl * nr + 1))
        check_all(api, int(nl), int(nr), l, r)


@pytest.mark.parametrize("a,b", [(1, 1), (2, 2), (2, 3), (17, 5), (300, 3), (3, 300), (64, 64)])
def test_complete_bipartite(api, a, b):
    l, r = gen.biclique(a, b)
    B = check_all(api, a, b, l, r)
    assert B == (a * (a - 1) // 2) * (b * (b - 1) // 2)


def test_dataset_table_biclique(api):
    # first row of the paper's dataset table: (10^4, 10)-biclique
    l, r = gen.biclique(10_000, 10)
    g = api.Graph(10_000, 10, l, r)
    assert g.exact() == 2_249_775_000
    assert g.sumsq == (1_000_000, 1_000_000_000)
    assert g.side_used() == 2
    cl, cr, ce = g.local()
    assert (cl == 9_999 * 45).all() and (cr == 9 * (10_000 * 9_999 // 2)).all()
    assert (ce == 9_999 * 9).all()


def test_empty_and_isolated(api):
    e = np.zeros(0, np.uint32)
    g = api.Graph(5, 7, e, e)
    assert g.exact() == 0
    cl, cr, ce = g.local()
    assert cl.tolist() == [0] * 5 and cr.tolist() == [0] * 7 and ce.size == 0
    # a single edge among many isolated vertices
    g = api.Graph(1000, 1000, np.array([999], np.uint32), np.array([0], np.uint32))
    assert g.exact() == 0


def test_errors(api):
    from paper_1801_00338_amd._lib import BfcError
    with pytest.raises(BfcError, match="DUP"):
        api.Graph(2, 2, np.array([0, 0], np.uint32), np.array([1, 1], np.uint32))
    with pytest.raises(BfcError, match="ID_RANGE"):
        api.Graph(2, 2, np.array([0, 2], np.uint32), np.array([1, 1], np.uint32))
    g = api.Graph(2, 2, np.array([0], np.uint32), np.array([1], np.uint32))
    with pytest.raises(BfcError, match="ARG"):
        g.exact(side=7)


def test_er_2k_3k_20k(api):
    w = gen.WORKLOADS["er_2k_3k_20k"]
    l, r = w.edges()
    check_all(api, w.nl, w.nr, l, r)


def test_chung_lu_small_hubs(api):
    # power-law graph with hub starts (degree >= 256 takes the wide path)
    nl, nr = 3000, 15000
    l, r = gen.chung_lu(nl, nr, 150_000, 2.1, 2.3, 2000, seed=7)
    check_all(api, nl, nr, l, r)


def test_many_windows(api):
    # more than two 2^16-rank windows on either side, sparse: exercises the
    # window walk, skipped windows and the segment boundaries
    nl, nr = 200_000, 150_000
    l, r = gen.chung_lu(nl, nr, 600_000, 2.2, 2.4, 5000, seed=11)
    check_all(api, nl, nr, l, r, local=False)
    g = api.Graph(nl, nr, l, r)
    cl, cr, ce = g.local()
    ol, orr = oracle.per_vertex(nl, nr, l, r)
    assert np.array_equal(cl, ol) and np.array_equal(cr, orr)
    assert np.array_equal(ce, oracle.per_edge(nl, nr, l, r))


def test_dense_windows_multi_round(api):
    # Starting from L (forced, side 1): 4000 starts of degree 50 whose
    # midpoints have ~2000 entries each, so one window holds far more 4-entry
    # groups than the workgroup has lanes (the full table clear path).  The
    # automatic side starts from R: 100 starts of degree ~2000 (wide path).
    rng = np.random.default_rng(5)
    nl, nr = 4000, 100
    l = np.repeat(np.arange(nl, dtype=np.uint32), 50)
    r = np.concatenate([rng.choice(nr, 50, replace=False) for _ in range(nl)]).astype(np.uint32)
    check_all(api, nl, nr, l, r)


def test_local_wide_table_modes(api):
    """Local counts of wide starts in both table modes: 16-bit counters over
    2^15-rank windows (255 < d_u <= 65535) and 32-bit counters over 2^14
    ranks (d_u > 65535), with starts spread over several table windows."""
    rng = np.random.default_rng(23)
    nl, nr = 150_000, 70_000
    parts_l, parts_r = [], []
    # hub L0 joined to every R vertex (degree 70,000 > 65,535)
    parts_l.append(np.zeros(nr, np.uint32))
    parts_r.append(np.arange(nr, dtype=np.uint32))
    # 40 L vertices of degree 300..5000 (the 16-bit mode), spread over the id range
    for i, d in enumerate(np.linspace(300, 5000, 40).astype(int)):
        parts_l.append(np.full(d, 1 + i * 3000, np.uint32))
        parts_r.append(rng.choice(nr, d, replace=False).astype(np.uint32))
    l = np.concatenate(parts_l)
    r = np.concatenate(parts_r)
    # sparse background: random edges among the other L vertices
    bl = rng.integers(1, nl, 200_000).astype(np.uint32)
    br = rng.integers(0, nr, 200_000).astype(np.uint32)
    key = np.unique(np.concatenate([l.astype(np.uint64) * nr + r,
                                    bl.astype(np.uint64) * nr + br]))
    l = (key // nr).astype(np.uint32)
    r = (key % nr).astype(np.uint32)
    g = api.Graph(nl, nr, l, r)
    assert g.side_used() == api.BFC_SIDE_L and g.max_degree[0] == nr
    print(f"case nl={nl} nr={nr} m={l.size}", flush=True)
    cl, cr, ce = g.local()
    ol, orr = oracle.per_vertex(nl, nr, l, r)
    assert np.array_equal(cl, ol) and np.array_equal(cr, orr)
    assert np.array_equal(ce, oracle.per_edge(nl, nr, l, r))
    assert g.exact() == oracle.exact(nl, nr, l, r)[0]


# ------------------------------------------------------------------ hash-table starts
OFF = 0xFFFFFFFF
HASH_TUNINGS = [
    dict(hash_small_max=OFF, hash_mid_max=OFF),          # dense windows only
    dict(),                                              # defaults
    dict(hash_mid_max=OFF, hash_max_density=1 << 30),          # small tables only
    dict(hash_small_max=OFF, hash_max_density=1 << 30),        # mid tables only
    dict(hash_passes=1, hash_max_density=1 << 30),             # one pass: full tables fall back
    dict(hash_passes=4, hash_max_density=1 << 30),             # every start in four partitions
    dict(hash_small_max=64, hash_mid_max=300, hash_max_density=1 << 30),
]


def _hash_graphs():
    rng = np.random.default_rng(42)
    out = []
    l, r = rand_graph(rng, 40, 50, 900)
    out.append(("random 40x50", 40, 50, l, r))
    nl, nr = 200_000, 150_000          # sparse ends spread over many windows
    l, r = gen.chung_lu(nl, nr, 600_000, 2.2, 2.4, 5000, seed=11)
    out.append(("chung_lu 200k/150k/600k", nl, nr, l, r))
    nl, nr = 20_000, 60_000            # power law with hubs: all four classes
    l, r = gen.chung_lu(nl, nr, 600_000, 2.1, 2.3, 5_000, seed=71)
    out.append(("chung_lu 20k/60k/600k", nl, nr, l, r))
    l, r = gen.biclique(40, 60)        # 60 midpoints, every start T = 60 * (rank above)
    out.append(("K_40,60", 40, 60, l, r))
    return out


@pytest.mark.parametrize("case", range(4))
def test_hash_classes_against_oracle(api, case):
    """The hash-table walk, the dense windows and the fallback of full tables
    all give the oracle's count, from both sides, under every class split."""
    name, nl, nr, l, r = _hash_graphs()[case]
    g = api.Graph(nl, nr, l, r)
    want = oracle.exact(nl, nr, l, r)[0]
    for t in HASH_TUNINGS:
        print(f"{name}: {t}", flush=True)
        assert g.exact_tuned(t) == want, t
        for side in (1, 2):
            assert g.exact_tuned(t, side=side) == want, (t, side)


def test_hash_full_table_falls_back(api):
    """A start whose single pass overflows the 1,024-slot table (2,001
    distinct end points, each reached once) is counted by the narrow walk
    instead; with automatic passes it fits in four partitions."""
    # L: u = 0, a_i = 1..1000, b_i = 1001..2000, u' = 2001 (all of degree 2);
    # R: x = 0, y = 1, z_i = 1 + i (shared by a_i and b_i)
    a = np.arange(1, 1001, dtype=np.uint32)
    b = np.arange(1001, 2001, dtype=np.uint32)
    z = np.arange(2, 1002, dtype=np.uint32)
    l = np.concatenate([[0, 0, 2001, 2001], a, a, b, b]).astype(np.uint32)
    r = np.concatenate([[0, 1, 0, 1], np.zeros(1000), z, np.ones(1000), z]).astype(np.uint32)
    nl, nr = 2002, 1002
    g = api.Graph(nl, nr, l, r)
    want = oracle.exact(nl, nr, l, r)[0]
    dense = 1 << 30                    # every start counts as sparse
    for t in (dict(hash_passes=1, hash_max_density=dense),
              dict(hash_passes=2, hash_max_density=dense), dict(hash_max_density=dense), {}):
        print(f"fallback case: {t}", flush=True)
        assert g.exact_tuned(t, side=1) == want, t
        assert g.exact_tuned(t, side=2) == want, t


# ------------------------------------------------------------------ hub starts split over workgroups
@pytest.mark.parametrize("case", ["windows", "hubs"])
def test_local_counts_with_split_hub_starts(api, case):
    """Local counts with hub starts cut into runs of counter windows walked by
    different workgroups (down to one window per part) equal the oracle's
    per-vertex and per-edge counts."""
    if case == "windows":
        nl, nr = 200_000, 150_000
        l, r = gen.chung_lu(nl, nr, 600_000, 2.2, 2.4, 5000, seed=11)
    else:
        nl, nr = 100_000, 60_000
        l, r = gen.chung_lu(nl, nr, 1_000_000, 2.1, 2.1, 20_000, seed=23)
    g = api.Graph(nl, nr, l, r)
    ol, orr = oracle.per_vertex(nl, nr, l, r)
    oe = oracle.per_edge(nl, nr, l, r)
    for split in (0, 1, 1000, 100_000):
        print(f"{case}: split {split}", flush=True)
        cl, cr, ce = g.local_split(split)
        assert np.array_equal(cl, ol), split
        assert np.array_equal(cr, orr), split
        assert np.array_equal(ce, oe), split
    # vertex counts only (no second look at the final counts)
    cl, cr, _ = g.local_split(1, edges=False)
    assert np.array_equal(cl, ol) and np.array_equal(cr, orr)


# ------------------------------------------------------------------ sparse hubs on a large side
def test_sparse_hubs_on_a_large_side(api):
    """Hub starts whose midpoints have short lists spread over a side of 2M
    ranks (62 to 123 counter windows): fewer wedges than (midpoint, window)
    pairs, so the wide walks take one-group pieces, and hubs past the
    register-cursor limit load a cursor only in the windows where it has
    entries.  Degrees 300 and 400 (register cursors), 700, 900 and 3,000
    (workspace cursors, 16-bit table) and 70,000 (32-bit table); whole and
    split into parts of few windows."""
    rng = np.random.default_rng(31)
    nl, nr = 2_000_000, 80_000
    parts_l, parts_r = [], []
    for i, d in enumerate((300, 400, 700, 900, 3000, 70_000)):
        parts_l.append(np.full(d, i * 333_331, np.uint32))
        parts_r.append(rng.choice(nr, d, replace=False).astype(np.uint32))
    bl = rng.integers(0, nl, 240_000).astype(np.uint64)
    br = rng.integers(0, nr, 240_000).astype(np.uint64)
    key = np.unique(np.concatenate([np.concatenate(parts_l).astype(np.uint64) * nr
                                    + np.concatenate(parts_r), bl * nr + br]))
    l = (key // nr).astype(np.uint32)
    r = (key % nr).astype(np.uint32)
    print(f"case nl={nl} nr={nr} m={l.size}", flush=True)
    g = api.Graph(nl, nr, l, r)
    assert g.side_used() == api.BFC_SIDE_L
    want = oracle.exact(nl, nr, l, r)[0]
    for side in (0, 1, 2):
        assert g.exact(side) == want, side
    ol, orr = oracle.per_vertex(nl, nr, l, r)
    oe = oracle.per_edge(nl, nr, l, r)
    for split in (0, 1, 5000):
        print(f"split {split}", flush=True)
        cl, cr, ce = g.local_split(split)
        assert np.array_equal(cl, ol), split
        assert np.array_equal(cr, orr), split
        assert np.array_equal(ce, oe), split
