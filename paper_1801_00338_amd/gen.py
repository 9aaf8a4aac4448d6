"""Seeded synthetic bipartite workloads.

This module only produces inputs: uint32 edge lists (l_ids, r_ids) of simple
bipartite graphs.  It holds none of the counting arithmetic, so both the HIP
path and the CPU oracle can be fed from it.

Two families stand in for the KONECT graphs of the paper's dataset table
(Sec. 2, "Networks and Experimental Setup"): uniform (Erdos-Renyi style)
bipartite graphs and Chung-Lu power-law bipartite graphs.  The paper removes
multi-edges and self loops; bipartite graphs have no self loops, and both
generators drop repeated (l, r) pairs.

Recipe (deterministic for a given seed; the sampler is gen_native.c, a
SplitMix64 stream with Walker alias tables):

* er(nl, nr, m, seed): endpoints drawn uniformly and independently on each
  side; the first m distinct pairs in draw order are kept.
* chung_lu(nl, nr, m, gamma_l, gamma_r, cap, seed): vertex i of a side of size
  n gets weight (i+1)^(-1/(gamma-1)); expected degrees m*w_i/sum(w) are capped
  at ``cap`` by iterated capping (the excess is redistributed proportionally
  over the uncapped vertices until none exceeds the cap); endpoints are drawn
  independently on each side with probability proportional to the capped
  expected degree, the first m distinct pairs in draw order are kept, and each
  side's ids are relabelled by a seeded random permutation so that hubs are
  not clustered at low ids.

Edges come back in draw order (not sorted), as uint32 numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

__all__ = ["er", "chung_lu", "capped_expected_degrees", "biclique",
           "disjoint_union", "Workload", "WORKLOADS", "make_workload", "build_native",
           "mlp_init", "batch_order", "training_graphs", "batch_specs", "batch_graphs"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen_native.c")
_LIB = os.path.join(_HERE, "libbfcgen.so")
_lib = None


def build_native(force: bool = True) -> str:
    """Compile the sampler with gcc (host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _native():
    global _lib
    if _lib is None:
        build_native(force=False)
        L = C.CDLL(_LIB)
        u32p = C.POINTER(C.c_uint32)
        dp = C.POINTER(C.c_double)
        L.gen_er.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64, u32p, u32p]
        L.gen_weighted.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, dp, dp, C.c_uint64,
                                   C.c_int, u32p, u32p]
        _lib = L
    return _lib


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


def _u32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def _check(rc):
    if rc == -2:
        raise ValueError("graph too dense: could not draw enough distinct edges")
    if rc == -3:
        raise ValueError("m exceeds |L|*|R|")
    if rc != 0:
        raise MemoryError("generator out of memory")


def er(nl: int, nr: int, m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Uniform bipartite graph with exactly m distinct edges."""
    if m > nl * nr:
        raise ValueError("m exceeds |L|*|R|")
    l = np.zeros(max(m, 1), np.uint32)
    r = np.zeros(max(m, 1), np.uint32)
    if m:
        _check(_native().gen_er(nl, nr, m, seed, _u32p(l), _u32p(r)))
    return l[:m], r[:m]


def chung_lu(nl: int, nr: int, m: int, gamma_l: float, gamma_r: float,
             cap: float, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Chung-Lu power-law bipartite graph with exactly m distinct edges."""
    if m > nl * nr:
        raise ValueError("m exceeds |L|*|R|")
    l = np.zeros(max(m, 1), np.uint32)
    r = np.zeros(max(m, 1), np.uint32)
    if m:
        el = np.ascontiguousarray(capped_expected_degrees(nl, m, gamma_l, min(cap, nr)))
        er_ = np.ascontiguousarray(capped_expected_degrees(nr, m, gamma_r, min(cap, nl)))
        dp = C.POINTER(C.c_double)
        _check(_native().gen_weighted(nl, nr, m, el.ctypes.data_as(dp), er_.ctypes.data_as(dp),
                                      seed, 1, _u32p(l), _u32p(r)))
    return l[:m], r[:m]


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
    "chung_lu_20m_80m_400m": Workload("chung_lu_20m_80m_400m", "chung_lu",
                                      20_000_000, 80_000_000, 400_000_000,
                                      2.1, 2.3, 100_000, seed=5),
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


# ---------------------------------------------------------------- learned sampling inputs
MLP_PARAMS = 4801     # W1[8][64], b1[64], W2[64][64], b2[64], w3[64], b3


def mlp_init(seed: int) -> np.ndarray:
    """Seeded initial parameters of the 8 -> 64 -> 64 -> 1 network (float32).

    Weights uniform in +-sqrt(6 / fan_in) (He), w3 in +-sqrt(3 / 64), biases 0.
    """
    rng = np.random.default_rng(seed)
    p = np.zeros(MLP_PARAMS, np.float32)
    p[0:512] = rng.uniform(-1, 1, 512) * math.sqrt(6 / 8)
    p[576:4672] = rng.uniform(-1, 1, 4096) * math.sqrt(6 / 64)
    p[4736:4800] = rng.uniform(-1, 1, 64) * math.sqrt(3 / 64)
    return p


def batch_order(seed: int, n: int, epoch: int) -> np.ndarray:
    """A seeded permutation of range(n) (uint32) for one epoch of mini-batches."""
    rng = np.random.default_rng([seed, epoch])
    return rng.permutation(n).astype(np.uint32)


def training_graphs(count: int, m_lo: int, m_hi: int, seed: int, ratio: float = 4.0,
                    mean_degree: float = 8.0, gamma_l: float = 2.1, gamma_r: float = 2.3):
    """``count`` Chung-Lu graphs with m log-spaced in [m_lo, m_hi] and |R| = ratio |L|.

    Mean degree 2m / (|L| + |R|) = ``mean_degree``; graph j uses seed
    (seed << 32) | (j + 1); the expected-degree cap is min(14 sqrt(m), |L| / 4)
    (14 sqrt(m) is 100k at 50M edges).  Returns a list of (nl, nr, l, r).
    """
    out = []
    ms = np.geomspace(m_lo, m_hi, count) if count > 1 else np.array([m_lo])
    for j, m in enumerate(ms):
        m = int(round(m))
        n = 2.0 * m / mean_degree
        nl = max(2, int(round(n / (1 + ratio))))
        nr = max(2, int(round(n - nl)))
        cap = max(2.0, min(100_000.0, 14.0 * math.sqrt(m), nl / 4))
        l, r = chung_lu(nl, nr, m, gamma_l, gamma_r, cap, (seed << 32) | (j + 1))
        out.append((nl, nr, l, r))
    return out


# ---------------------------------------------------------------- batches of uneven graphs
def batch_specs(count: int, m_lo: int, m_hi: int, seed: int = 3):
    """Parameters of a batch of uneven graphs (no edges drawn yet).

    Per graph q (one numpy stream seeded with ``seed``): m log-uniform in
    [m_lo, m_hi]; |L|:|R| = rho uniform in [0.2, 5]; mean degree 2m / (|L| +
    |R|) log-uniform in [4, 32]; |L| = round(n rho / (1 + rho)), with |L| |R|
    >= 4m enforced; the first half of the graphs Erdos-Renyi, the second half
    Chung-Lu with one gamma uniform in [2.0, 2.8] for both sides and the
    expected-degree cap min(100k, sqrt(|L| |R|)) raised where needed to
    exceed m / min(|L|, |R|).  Graph q draws its edges with seed
    (seed << 32) | q.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for q in range(count):
        m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        rho = rng.uniform(0.2, 5.0)
        d = math.exp(rng.uniform(math.log(4), math.log(32)))
        gamma = rng.uniform(2.0, 2.8)
        n = 2.0 * m / d
        nl = max(2, int(round(n * rho / (1 + rho))))
        nr = max(2, int(round(n - nl)))
        while nl * nr < 4 * m:
            nl += max(1, nl // 8)
            nr += max(1, nr // 8)
        kind = "er" if q < count // 2 else "chung_lu"
        cap = min(100_000.0, math.sqrt(nl * nr))
        cap = max(cap, 1.01 * m / min(nl, nr), 2.0)
        specs.append(dict(q=q, kind=kind, nl=nl, nr=nr, m=m, gamma=gamma, cap=cap,
                          seed=(seed << 32) | q))
    return specs


def batch_graphs(count: int, m_lo: int, m_hi: int, seed: int = 3):
    """The graphs of ``batch_specs``: a list of (nl, nr, l, r)."""
    out = []
    for sp in batch_specs(count, m_lo, m_hi, seed):
        if sp["kind"] == "er":
            l, r = er(sp["nl"], sp["nr"], sp["m"], sp["seed"])
        else:
            l, r = chung_lu(sp["nl"], sp["nr"], sp["m"], sp["gamma"], sp["gamma"], sp["cap"],
                            sp["seed"])
        out.append((sp["nl"], sp["nr"], l, r))
    return out
