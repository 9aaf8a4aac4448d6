"""Brute-force enumerations for tiny graphs -- TEST INFRASTRUCTURE ONLY.

These are independent of the C oracle (no shared code): they enumerate the
definitions of Sec. 2 of the paper directly.

* A butterfly is a 2x2 biclique {a, b} x {x, y} (a, b in L; x, y in R) with
  all four edges present.
* The per-vertex count B_v is the number of butterflies containing v; the
  per-edge count B_e the number containing e.
* Pairs of distinct butterflies fall into the types 0v, 1v, 2v, 1e, 1w of the
  variance analysis of Sec. 5.1 (shared vertices / edges / a wedge).
"""
from __future__ import annotations

from itertools import combinations


def butterflies(nl, nr, l, r):
    """All butterflies as (a, b, x, y) with a < b in L and x < y in R."""
    edges = set(zip((int(a) for a in l), (int(b) for b in r)))
    nbr = {}
    for a, x in edges:
        nbr.setdefault(a, set()).add(x)
    out = []
    left = sorted(nbr)
    for i, a in enumerate(left):
        for b in left[i + 1:]:
            common = sorted(nbr[a] & nbr[b])
            for x, y in combinations(common, 2):
                out.append((a, b, x, y))
    return out


def butterflies_quadruples(nl, nr, l, r):
    """Count by checking every 2x2 vertex quadruple (slowest, most literal)."""
    edges = set(zip((int(a) for a in l), (int(b) for b in r)))
    n = 0
    for a, b in combinations(range(nl), 2):
        for x, y in combinations(range(nr), 2):
            if (a, x) in edges and (a, y) in edges and (b, x) in edges and (b, y) in edges:
                n += 1
    return n


def per_vertex(nl, nr, l, r):
    cl = [0] * nl
    cr = [0] * nr
    for a, b, x, y in butterflies(nl, nr, l, r):
        cl[a] += 1
        cl[b] += 1
        cr[x] += 1
        cr[y] += 1
    return cl, cr


def per_edge(nl, nr, l, r):
    """Per-edge counts in input order."""
    idx = {(int(a), int(x)): i for i, (a, x) in enumerate(zip(l, r))}
    ce = [0] * len(idx)
    for a, b, x, y in butterflies(nl, nr, l, r):
        for e in ((a, x), (a, y), (b, x), (b, y)):
            ce[idx[e]] += 1
    return ce


def pair_types(nl, nr, l, r):
    """Counts of unordered pairs of distinct butterflies by type.

    Type of a pair: number of shared vertices and shared edges.
      0v: no shared vertex; 1v: one shared vertex;
      2v: two shared vertices, no shared edge;
      1e: two shared vertices joined by a shared edge;
      1w: three shared vertices (two shared edges forming a wedge).
    """
    bf = butterflies(nl, nr, l, r)
    verts = []
    edges = []
    for a, b, x, y in bf:
        verts.append({("L", a), ("L", b), ("R", x), ("R", y)})
        edges.append({(a, x), (a, y), (b, x), (b, y)})
    t = {"0v": 0, "1v": 0, "2v": 0, "1e": 0, "1w": 0}
    for i in range(len(bf)):
        for j in range(i + 1, len(bf)):
            sv = len(verts[i] & verts[j])
            se = len(edges[i] & edges[j])
            if sv == 0:
                t["0v"] += 1
            elif sv == 1:
                t["1v"] += 1
            elif sv == 2 and se == 0:
                t["2v"] += 1
            elif sv == 2 and se == 1:
                t["1e"] += 1
            elif sv == 3 and se == 2:
                t["1w"] += 1
            else:
                raise AssertionError(f"unexpected pair type: {sv} vertices, {se} edges")
    return t


def ebfc_as_printed(nl, nr, l, r, e):
    """eBFC with the fold exactly as printed in Sec. 4.2: sum C(C[x], 2).

    Kept only to show, on K_{2,3}, that this fold disagrees with the
    definition of the per-edge count.
    """
    u, v = int(l[e]), int(r[e])
    nbr_l, nbr_r = {}, {}
    for a, x in zip(l, r):
        nbr_l.setdefault(int(a), set()).add(int(x))
        nbr_r.setdefault(int(x), set()).add(int(a))
    C = {}
    for w in nbr_l.get(u, ()):
        for x in nbr_r.get(w, ()):
            if x in nbr_r.get(v, set()) and x != u:
                C[x] = C.get(x, 0) + 1
    return sum(c * (c - 1) // 2 for c in C.values())
