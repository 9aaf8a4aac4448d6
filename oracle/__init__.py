"""CPU oracle for butterfly counting -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it and
shares no code with it.

``bfc_oracle.c`` (plain C, built into ``liboracle_bfc.so`` next to it) holds
the reference computations; ``brute`` holds pure-Python enumerations for tiny
graphs that pin the C oracle.  Functions take numpy uint32 edge arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_bfc.so")

ERRORS = {0: "ok", -1: "bad argument", -2: "id out of range", -3: "duplicate edge",
          -4: "out of memory", -5: "bad probabilities", -6: "overflow"}

TAG_ESPAR = 0x45535052
TAG_COLOR = 0x434C5253
TAG_VDRAW = 0x56445257
TAG_EDRAW = 0x45445257
TAG_WDRAW = 0x57445257
TAG_FAST = 0x46454243


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-Wall", "-shared", "-fPIC",
                               "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        u32p, u64p, dp = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        g = [C.c_uint32, C.c_uint32, C.c_uint64, u32p, u32p]
        L.orc_exact.argtypes = g + [C.c_int, u64p, u64p, ip]
        L.orc_exact_range.argtypes = g + [C.c_int, C.c_uint64, C.c_uint64, u64p, u64p, ip]
        L.orc_degree_stats.argtypes = g + [u64p, u64p, u64p, u64p]
        L.orc_per_vertex.argtypes = g + [u64p, u64p]
        L.orc_vbfc.argtypes = g + [C.c_int, C.c_uint32, u64p]
        L.orc_per_edge.argtypes = g + [u64p]
        L.orc_ebfc.argtypes = g + [C.c_uint64, u64p]
        L.orc_espar.argtypes = g + [C.c_double, C.c_uint64, u64p, dp, u64p]
        L.orc_clrspar.argtypes = g + [C.c_uint32, C.c_uint64, u64p, dp, u64p]
        L.orc_vsamp.argtypes = g + [dp, C.c_uint64, C.c_uint64, u32p, u64p, dp]
        L.orc_esamp.argtypes = g + [dp, C.c_uint64, C.c_uint64, u64p, u64p, dp]
        L.orc_esamp_fast.argtypes = g + [dp, C.c_uint64, C.c_uint32, C.c_uint64, u64p, u32p, dp]
        L.orc_fast_ebfc_pairs.argtypes = g + [C.c_uint64, u64p]
        L.orc_wsamp.argtypes = g + [C.c_uint64, C.c_uint64, u32p, u32p, u64p, dp]
        L.orc_wedges.argtypes = g + [u64p, C.c_uint64, u32p, u32p, u64p, u64p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_color.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_color.restype = C.c_uint32
        L.orc_uniform_below.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint64, u64p]
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads over start vertices for exact, exact_range, per_vertex and
    per_edge (1 = in order on the calling thread, the default).  Results do
    not depend on it.  Returns the setting in force."""
    lib().orc_set_threads(int(n))
    return int(lib().orc_get_threads())


def _edges(l, r):
    l = np.ascontiguousarray(l, dtype=np.uint32)
    r = np.ascontiguousarray(r, dtype=np.uint32)
    if l.shape != r.shape:
        raise ValueError("l and r differ in length")
    return l, r


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


def _g(nl, nr, l, r):
    return [C.c_uint32(nl), C.c_uint32(nr), C.c_uint64(l.size), _p(l, C.c_uint32), _p(r, C.c_uint32)]


def exact(nl, nr, l, r, side=0):
    """ExactBFC: returns (butterflies, wedges visited, side used 1=L/2=R)."""
    l, r = _edges(l, r)
    t, w, s = C.c_uint64(), C.c_uint64(), C.c_int()
    _check(lib().orc_exact(*_g(nl, nr, l, r), side, C.byref(t), C.byref(w), C.byref(s)))
    return t.value, w.value, s.value


def exact_range(nl, nr, l, r, side, lo, hi):
    """ExactBFC over the starts [lo, hi) of the chosen side only."""
    l, r = _edges(l, r)
    t, w, s = C.c_uint64(), C.c_uint64(), C.c_int()
    _check(lib().orc_exact_range(*_g(nl, nr, l, r), side, lo, hi, C.byref(t), C.byref(w),
                                 C.byref(s)))
    return t.value, w.value, s.value


def degree_stats(nl, nr, l, r):
    l, r = _edges(l, r)
    a, b, c, d = C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_uint64()
    _check(lib().orc_degree_stats(*_g(nl, nr, l, r), C.byref(a), C.byref(b), C.byref(c),
                                  C.byref(d)))
    return a.value, b.value, c.value, d.value


def per_vertex(nl, nr, l, r):
    l, r = _edges(l, r)
    cl = np.zeros(max(nl, 1), np.uint64)
    cr = np.zeros(max(nr, 1), np.uint64)
    _check(lib().orc_per_vertex(*_g(nl, nr, l, r), _p(cl, C.c_uint64), _p(cr, C.c_uint64)))
    return cl[:nl], cr[:nr]


def vbfc(nl, nr, l, r, side, v):
    l, r = _edges(l, r)
    o = C.c_uint64()
    _check(lib().orc_vbfc(*_g(nl, nr, l, r), side, v, C.byref(o)))
    return o.value


def per_edge(nl, nr, l, r):
    l, r = _edges(l, r)
    ce = np.zeros(max(l.size, 1), np.uint64)
    _check(lib().orc_per_edge(*_g(nl, nr, l, r), _p(ce, C.c_uint64)))
    return ce[:l.size]


def ebfc(nl, nr, l, r, e):
    l, r = _edges(l, r)
    o = C.c_uint64()
    _check(lib().orc_ebfc(*_g(nl, nr, l, r), e, C.byref(o)))
    return o.value


def espar(nl, nr, l, r, p, seed):
    """Returns (beta, estimate, kept edge count)."""
    l, r = _edges(l, r)
    b, e, k = C.c_uint64(), C.c_double(), C.c_uint64()
    _check(lib().orc_espar(*_g(nl, nr, l, r), p, seed, C.byref(b), C.byref(e), C.byref(k)))
    return b.value, e.value, k.value


def clrspar(nl, nr, l, r, ncolors, seed):
    """Returns (beta, estimate, kept edge count)."""
    l, r = _edges(l, r)
    b, e, k = C.c_uint64(), C.c_double(), C.c_uint64()
    _check(lib().orc_clrspar(*_g(nl, nr, l, r), ncolors, seed, C.byref(b), C.byref(e),
                             C.byref(k)))
    return b.value, e.value, k.value


def vsamp(nl, nr, l, r, k, seed, probs=None):
    """Returns (ids[k] (global: L ids then nl + R id), counts[k], estimate)."""
    l, r = _edges(l, r)
    ids = np.zeros(k, np.uint32)
    cnt = np.zeros(k, np.uint64)
    est = C.c_double()
    pp = None
    if probs is not None:
        probs = np.ascontiguousarray(probs, dtype=np.float64)
        pp = _p(probs, C.c_double)
    _check(lib().orc_vsamp(*_g(nl, nr, l, r), pp, k, seed, _p(ids, C.c_uint32),
                           _p(cnt, C.c_uint64), C.byref(est)))
    return ids, cnt, est.value


def esamp(nl, nr, l, r, k, seed, probs=None):
    """Returns (edge indices[k], counts[k], estimate)."""
    l, r = _edges(l, r)
    eids = np.zeros(k, np.uint64)
    cnt = np.zeros(k, np.uint64)
    est = C.c_double()
    pp = None
    if probs is not None:
        probs = np.ascontiguousarray(probs, dtype=np.float64)
        pp = _p(probs, C.c_double)
    _check(lib().orc_esamp(*_g(nl, nr, l, r), pp, k, seed, _p(eids, C.c_uint64),
                           _p(cnt, C.c_uint64), C.byref(est)))
    return eids, cnt, est.value


def esamp_fast(nl, nr, l, r, k, alpha, seed, probs=None):
    """ESamp with Fast-eBFC (Sec. 5.5): returns (edge indices[k], hits[k], estimate)."""
    l, r = _edges(l, r)
    eids = np.zeros(k, np.uint64)
    hits = np.zeros(k, np.uint32)
    est = C.c_double()
    pp = None
    if probs is not None:
        probs = np.ascontiguousarray(probs, dtype=np.float64)
        pp = _p(probs, C.c_double)
    _check(lib().orc_esamp_fast(*_g(nl, nr, l, r), pp, k, alpha, seed, _p(eids, C.c_uint64),
                                _p(hits, C.c_uint32), C.byref(est)))
    return eids, hits, est.value


def fast_ebfc_pairs(nl, nr, l, r, e):
    """Hitting neighbour pairs of input edge e over all d_a * d_x picks."""
    l, r = _edges(l, r)
    out = C.c_uint64()
    _check(lib().orc_fast_ebfc_pairs(*_g(nl, nr, l, r), e, C.byref(out)))
    return out.value


def wsamp(nl, nr, l, r, k, seed):
    """WSamp (Sec. 5.3): returns (midpoints[k], ends[k, 2], counts[k], estimate); ids global."""
    l, r = _edges(l, r)
    mids = np.zeros(k, np.uint32)
    ends = np.zeros((k, 2), np.uint32)
    cnt = np.zeros(k, np.uint64)
    est = C.c_double()
    _check(lib().orc_wsamp(*_g(nl, nr, l, r), k, seed, _p(mids, C.c_uint32),
                           _p(ends, C.c_uint32), _p(cnt, C.c_uint64), C.byref(est)))
    return mids, ends, cnt, est.value


def wedges(nl, nr, l, r, t=None):
    """Decode wedge numbers t (default: all): (midpoints, ends, counts, W)."""
    l, r = _edges(l, r)
    W = C.c_uint64()
    if t is None:
        _check(lib().orc_wedges(*_g(nl, nr, l, r), None, 0, None, None, None, C.byref(W)))
        t = np.arange(W.value, dtype=np.uint64)
    t = np.ascontiguousarray(t, dtype=np.uint64)
    mids = np.zeros(t.size, np.uint32)
    ends = np.zeros((t.size, 2), np.uint32)
    cnt = np.zeros(t.size, np.uint64)
    _check(lib().orc_wedges(*_g(nl, nr, l, r), _p(t, C.c_uint64), t.size, _p(mids, C.c_uint32),
                            _p(ends, C.c_uint32), _p(cnt, C.c_uint64), C.byref(W)))
    return mids, ends, cnt, W.value


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(o, C.c_uint32))
    return o


def color(seed, side, v, ncolors):
    return int(lib().orc_color(seed, side, v, ncolors))


def uniform_below(seed, a, b, tag, n):
    o = C.c_uint64()
    _check(lib().orc_uniform_below(seed, a, b, tag, n, C.byref(o)))
    return o.value
