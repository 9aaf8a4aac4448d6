"""Seeded synthetic bipartite workloads.

This module only produces inputs: uint32 edge lists (l_ids, r_ids) of simple
bipartite graphs.  It holds none of the counting arithmetic, so both the HIP
path and the CPU oracle can be fed from it.

Two families stand in for the KONECT graphs of the paper's dataset table
(Sec. 2, "Networks and Experimental Setup"): uniform (Erdos-Renyi style)
bipartite graphs and Chung-Lu power-law bipartite graphs.  The paper removes
multi-edges and self loops; bipartite graphs have no self loops, and both
generators drop duplicate (l, r) pairs.

Recipe (fixed, deterministic for a given seed, numpy PCG64 stream):

* ER(nl, nr, m, seed): endpoints drawn uniformly and independently on each
  side; the first m distinct pairs in draw order are kept.
* Chung-Lu(nl, nr, m, gamma_l, gamma_r, cap, seed): vertex i of a side of size
  n gets weight (i+1)^(-1/(gamma-1)); expected degrees m*w_i/sum(w) are capped
  at ``cap`` by iterated capping (the excess is redistributed proportionally
  over the uncapped vertices until no vertex exceeds the cap); endpoints are
  then drawn independently on each side with probability proportional to the
  capped expected degree, and the first m distinct pairs in draw order are
  kept.  Finally each side's ids are relabelled by a seeded random permutation
  so that hubs are not clustered at low ids.

Edges come back in draw order (not sorted), as uint32 numpy arrays.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["er", "chung_lu", "capped_expected_degrees", "biclique",
           "disjoint_union", "Workload", "WORKLOADS", "make_workload"]


def capped_expected_degrees(n: int, m: int, gamma: float, cap: float) -> np.ndarray:
    """Expected degrees of a Chung-Lu side, rank-ordered, capped at ``cap``."""
    if n <= 0:
        return np.zeros(0, dtype=np.float64)
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (gamma - 1.0))
    e = w * (m / w.sum())
    cap = float(cap)
    if cap * n < m:
        raise ValueError("cap too small for the requested edge count")
    fixed = np.zeros(n, dtype=bool)
    for _ in range(64):
        over = (e > cap) & ~fixed
        if not over.any():
            break
        fixed |= over
        e[fixed] = cap
        rest = m - cap * fixed.sum()
        free = ~fixed
        e[free] *= rest / e[free].sum()
    return e


def _first_distinct(rng, m: int, draw, nr: int) -> tuple[np.ndarray, np.ndarray]:
    """Draw (l, r) batches from ``draw`` until m distinct pairs exist; keep the
    first m distinct ones in draw order."""
    keys = np.zeros(0, dtype=np.uint64)
    have = 0
    batches = []
    while True:
        need = m - have
        size = int(need * 1.15) + 4096
        l, r = draw(size)
        batches.append(l.astype(np.uint64) * np.uint64(nr) + r.astype(np.uint64))
        keys = np.concatenate(batches) if len(batches) > 1 else batches[0]
        batches = [keys]
        _, first = np.unique(keys, return_index=True)
        have = first.size
        if have >= m:
            first.sort()
            sel = keys[first[:m]]
            l_out = (sel // np.uint64(nr)).astype(np.uint32)
            r_out = (sel % np.uint64(nr)).astype(np.uint32)
            return l_out, r_out
        if len(keys) > 64 * max(m, 1) + 10**6:
            raise ValueError("graph too dense for the requested edge count")


def er(nl: int, nr: int, m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Uniform bipartite graph with exactly m distinct edges."""
    if m > nl * nr:
        raise ValueError("m exceeds |L|*|R|")
    if m == 0:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    rng = np.random.Generator(np.random.PCG64(seed))

    def draw(size):
        return (rng.integers(0, nl, size, dtype=np.int64),
                rng.integers(0, nr, size, dtype=np.int64))

    return _first_distinct(rng, m, draw, nr)


def chung_lu(nl: int, nr: int, m: int, gamma_l: float, gamma_r: float,
             cap: float, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Chung-Lu power-law bipartite graph with exactly m distinct edges."""
    if m == 0:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    cap_l = min(cap, nr)
    cap_r = min(cap, nl)
    el = capped_expected_degrees(nl, m, gamma_l, cap_l)
    er_ = capped_expected_degrees(nr, m, gamma_r, cap_r)
    cl = np.cumsum(el)
    cr = np.cumsum(er_)
    rng = np.random.Generator(np.random.PCG64(seed))

    def draw(size):
        ul = rng.random(size) * cl[-1]
        ur = rng.random(size) * cr[-1]
        li = np.minimum(np.searchsorted(cl, ul, side="right"), nl - 1)
        ri = np.minimum(np.searchsorted(cr, ur, side="right"), nr - 1)
        return li, ri

    l, r = _first_distinct(rng, m, draw, nr)
    perm_l = rng.permutation(nl).astype(np.uint32)
    perm_r = rng.permutation(nr).astype(np.uint32)
    return perm_l[l], perm_r[r]


def biclique(a: int, b: int) -> tuple[np.ndarray, np.ndarray]:
    """Complete bipartite K_{a,b}: every left id joined to every right id."""
    l = np.repeat(np.arange(a, dtype=np.uint32), b)
    r = np.tile(np.arange(b, dtype=np.uint32), a)
    return l, r


def disjoint_union(parts):
    """Disjoint union of (nl, nr, l, r) parts -> (nl, nr, l, r)."""
    nl = nr = 0
    ls, rs = [], []
    for pnl, pnr, l, r in parts:
        ls.append(np.asarray(l, np.uint64) + nl)
        rs.append(np.asarray(r, np.uint64) + nr)
        nl += pnl
        nr += pnr
    return (nl, nr, np.concatenate(ls).astype(np.uint32),
            np.concatenate(rs).astype(np.uint32))


class Workload:
    """A named synthetic graph: sizes plus how to draw it."""

    def __init__(self, name, kind, nl, nr, m, gamma_l=None, gamma_r=None,
                 cap=100_000, seed=0):
        self.name, self.kind = name, kind
        self.nl, self.nr, self.m = nl, nr, m
        self.gamma_l, self.gamma_r, self.cap, self.seed = gamma_l, gamma_r, cap, seed

    def edges(self):
        if self.kind == "er":
            return er(self.nl, self.nr, self.m, self.seed)
        return chung_lu(self.nl, self.nr, self.m, self.gamma_l, self.gamma_r,
                        self.cap, self.seed)

    def describe(self):
        d = {"workload": self.name, "generator": self.kind, "n_left": self.nl,
             "n_right": self.nr, "n_edges": self.m, "seed": self.seed}
        if self.kind != "er":
            d.update(gamma_left=self.gamma_l, gamma_right=self.gamma_r,
                     max_expected_degree=self.cap)
        return d


# The paper-shaped synthetic workloads (seed = workload number).
WORKLOADS = {
    "er_2k_3k_20k": Workload("er_2k_3k_20k", "er", 2_000, 3_000, 20_000, seed=1),
    "chung_lu_1m_5m_50m": Workload("chung_lu_1m_5m_50m", "chung_lu", 1_000_000,
                                   5_000_000, 50_000_000, 2.1, 2.3, 100_000, seed=2),
    "chung_lu_10m_30m_100m": Workload("chung_lu_10m_30m_100m", "chung_lu",
                                      10_000_000, 30_000_000, 100_000_000,
                                      2.2, 2.4, 100_000, seed=4),
}


def make_workload(name: str) -> Workload:
    return WORKLOADS[name]


def scaled_chung_lu(scale: float, seed: int = 2):
    """The 1M/5M/50M Chung-Lu shape shrunk by ``scale`` (cap scaled too)."""
    nl = max(2, int(round(1_000_000 * scale)))
    nr = max(2, int(round(5_000_000 * scale)))
    m = max(1, int(round(50_000_000 * scale)))
    cap = max(2.0, 100_000 * math.sqrt(scale))
    return nl, nr, chung_lu(nl, nr, m, 2.1, 2.3, cap, seed)
