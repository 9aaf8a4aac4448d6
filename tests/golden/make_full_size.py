"""Write tests/golden/full_size.json: oracle results at the full workload sizes.

Only the CPU oracle (``oracle/``) computes these values; the seeded generator
(``paper_1801_00338_amd.gen``, which holds none of the counting arithmetic)
supplies the inputs.  For every graph the file also keeps the SHA-256 of its
edge arrays, so a test can tell a changed generator from a changed count.

Entries (ExactBFC, Sec. 4; local counts, Sec. 4.2 and Eq. (2)):

* chung_lu_1m_5m_50m: total, wedges, start side, and SHA-256 of the per-vertex
  counts (L then R, little-endian uint64) and of the per-edge counts (uint64, in
  the generator's edge order), with their sums;
* chung_lu_10m_30m_100m and chung_lu_20m_80m_400m: total, wedges, start side;
* batch_1024: the totals and start sides of the 1,024 uneven graphs
  (m log-uniform in [1k, 2M], generator seed 3).

Usage: python tests/golden/make_full_size.py [names...] (default: all).  Runs
the oracle with one thread per host core; the whole set takes about an hour on
eight cores (the per-vertex counts of the 50M-edge graph walk both sides).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1801_00338_amd import gen  # noqa: E402

OUT = os.path.join(HERE, "full_size.json")
ALL = ["batch_1024", "chung_lu_10m_30m_100m", "chung_lu_1m_5m_50m", "chung_lu_20m_80m_400m"]


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


def single(name, local):
    w = gen.WORKLOADS[name]
    t = time.time()
    l, r = w.edges()
    print(f"{name}: generated m={l.size} in {time.time() - t:.0f} s", flush=True)
    d = {"input": w.describe(), "edges_sha256": edge_sha(l, r)}
    t = time.time()
    b, wedges, side = oracle.exact(w.nl, w.nr, l, r)
    d.update(total=b, wedges=wedges, side="L" if side == 1 else "R")
    print(f"{name}: B={b} W={wedges} in {time.time() - t:.0f} s", flush=True)
    if local:
        t = time.time()
        ce = oracle.per_edge(w.nl, w.nr, l, r)
        d.update(per_edge_sha256=u64_sha(ce), per_edge_sum=int(ce.sum(dtype=np.uint64)))
        print(f"{name}: per-edge in {time.time() - t:.0f} s", flush=True)
        t = time.time()
        cl, cr = oracle.per_vertex(w.nl, w.nr, l, r)
        d.update(per_vertex_sha256=u64_sha(cl, cr),
                 per_vertex_sum_l=int(cl.sum(dtype=np.uint64)),
                 per_vertex_sum_r=int(cr.sum(dtype=np.uint64)))
        print(f"{name}: per-vertex in {time.time() - t:.0f} s", flush=True)
    return d


def batch():
    t = time.time()
    graphs = gen.batch_graphs(1024, 1_000, 2_000_000, seed=3)
    print(f"batch_1024: generated in {time.time() - t:.0f} s", flush=True)
    h = hashlib.sha256()
    totals, sides = [], []
    t = time.time()
    for nl, nr, l, r in graphs:
        h.update(edge_sha(l, r).encode())
        b, _, s = oracle.exact(nl, nr, l, r)
        totals.append(b)
        sides.append("L" if s == 1 else "R")
    print(f"batch_1024: counted in {time.time() - t:.0f} s", flush=True)
    return {"input": {"count": 1024, "m_lo": 1_000, "m_hi": 2_000_000, "seed": 3},
            "edges_sha256": h.hexdigest(), "totals": totals, "sides": sides}


def main(names):
    print("oracle threads:", oracle.set_threads(os.cpu_count() or 1), flush=True)
    for name in names:
        if name == "batch_1024":
            d = batch()
        else:
            d = single(name, local=(name == "chung_lu_1m_5m_50m"))
        cur = {}
        if os.path.exists(OUT):
            with open(OUT) as f:
                cur = json.load(f)
        cur[name] = d
        tmp = OUT + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cur, f, indent=1, sort_keys=True)
            f.write("\n")
        os.replace(tmp, OUT)
        print(f"{name}: written", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ALL)
