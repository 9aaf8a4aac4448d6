"""Python front end of the HIP library.

PyTorch supplies device memory (tensors) and streams; the library does every
step of the computation.  Device buffers are kept alive by the objects that
hand their pointers to the library.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import BFC_SIDE_AUTO, BFC_SIDE_L, BFC_SIDE_R, check, lib  # noqa: F401


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _bytes(n, device):
    return torch.empty(max(int(n), 256), dtype=torch.uint8, device=device)


def to_device_u32(a, device="cuda"):
    """numpy/torch uint32 ids -> contiguous device tensor (int32 storage)."""
    if isinstance(a, torch.Tensor):
        t = a
        if t.dtype == torch.uint32:
            t = t.view(torch.int32)
        elif t.dtype != torch.int32:
            t = t.to(torch.int32)
        return t.to(device).contiguous()
    arr = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(arr.view(np.int32)).to(device)


class Graph:
    """A bipartite graph resident in device memory (both CSRs, rank order)."""

    def __init__(self, n_left, n_right, l, r, device="cuda", stream=None, parts=None):
        """``parts`` = (part_l, part_r) device uint32 offsets: rank by (part, degree, id)."""
        L = lib()
        self.device = torch.device(device)
        dl = to_device_u32(l, self.device)
        dr = to_device_u32(r, self.device)
        if dl.numel() != dr.numel():
            raise ValueError("l and r differ in length")
        m = dl.numel()
        sz = C.c_size_t()
        check(L.bfc_graph_storage_size(n_left, n_right, m, C.byref(sz)), "storage size")
        self.storage = _bytes(sz.value, self.device)
        check(L.bfc_graph_build_ws_size(n_left, n_right, m, C.byref(sz)), "build ws size")
        ws = _bytes(sz.value, self.device)
        self.g = _lib.bfc_graph()
        if parts is None:
            check(L.bfc_graph_build(n_left, n_right, m, C.c_void_p(dl.data_ptr()),
                                    C.c_void_p(dr.data_ptr()),
                                    C.c_void_p(self.storage.data_ptr()), self.storage.numel(),
                                    C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                                    C.byref(self.g)), "graph build")
        else:
            pl, pr = parts
            check(L.bfc_graph_build_parts(n_left, n_right, m, C.c_void_p(dl.data_ptr()),
                                          C.c_void_p(dr.data_ptr()), pl.numel() - 1,
                                          C.c_void_p(pl.data_ptr()), C.c_void_p(pr.data_ptr()),
                                          C.c_void_p(self.storage.data_ptr()),
                                          self.storage.numel(), C.c_void_p(ws.data_ptr()),
                                          ws.numel(), _stream(stream), C.byref(self.g)),
                  "graph build (parts)")
        del ws
        self.n_left, self.n_right, self.n_edges = n_left, n_right, m
        self._ws = None

    # -------------------------------------------------------------- stats
    @property
    def sumsq(self):
        return self.g.sumsq_l, self.g.sumsq_r

    @property
    def max_degree(self):
        return self.g.max_deg_l, self.g.max_deg_r

    def side_used(self, side=BFC_SIDE_AUTO):
        rc = lib().bfc_side_used(C.byref(self.g), side)
        if rc < 0:
            check(rc, "side")
        return rc

    def wedges(self, side=BFC_SIDE_AUTO):
        w = C.c_uint64()
        check(lib().bfc_wedges(C.byref(self.g), side, C.byref(w)), "wedges")
        return w.value

    def workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = _bytes(nbytes, self.device)
        return self._ws

    # -------------------------------------------------------------- exact
    def exact_ws_size(self, side=BFC_SIDE_AUTO):
        sz = C.c_size_t()
        check(lib().bfc_exact_ws_size(C.byref(self.g), side, C.byref(sz)), "exact ws size")
        return sz.value

    def exact_async(self, out, side=BFC_SIDE_AUTO, stream=None):
        """Queue the exact count; out is a 1-element int64 device tensor."""
        ws = self.workspace(self.exact_ws_size(side))
        check(lib().bfc_exact(C.byref(self.g), side, C.c_void_p(out.data_ptr()),
                              C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "exact")
        return out

    def exact_plan(self, side=BFC_SIDE_AUTO, stream=None):
        ws = self.workspace(self.exact_ws_size(side))
        check(lib().bfc_exact_plan(C.byref(self.g), side, C.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream(stream)), "exact plan")

    def exact_count(self, out, side=BFC_SIDE_AUTO, stream=None):
        """Queue the count on a workspace planned by exact_plan for this side."""
        ws = self.workspace(self.exact_ws_size(side))
        check(lib().bfc_exact_count(C.byref(self.g), side, C.c_void_p(out.data_ptr()),
                                    C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)),
              "exact count")
        return out

    def exact(self, side=BFC_SIDE_AUTO):
        out = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.exact_async(out, side)
        torch.cuda.synchronize(self.device)
        return int(out.cpu().numpy().view(np.uint64)[0])

    # -------------------------------------------------------------- local
    def local_ws_size(self):
        sz = C.c_size_t()
        check(lib().bfc_local_ws_size(C.byref(self.g), C.byref(sz)), "local ws size")
        return sz.value

    def local_async(self, cnt_l=None, cnt_r=None, cnt_e=None, stream=None):
        ws = self.workspace(self.local_ws_size())
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        check(lib().bfc_local(C.byref(self.g), ptr(cnt_l), ptr(cnt_r), ptr(cnt_e),
                              C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "local")

    def local_split(self, split_wedges, vertices=True, edges=True):
        """bfc_local_split: local counts with hub starts cut into parts of about
        ``split_wedges`` wedges (same results as local())."""
        d = self.device
        sz = C.c_size_t()
        check(lib().bfc_local_split_ws_size(C.byref(self.g), split_wedges, C.byref(sz)),
              "local split ws size")
        ws = _bytes(sz.value, d)
        cl = torch.zeros(max(self.n_left, 1), dtype=torch.int64, device=d) if vertices else None
        cr = torch.zeros(max(self.n_right, 1), dtype=torch.int64, device=d) if vertices else None
        ce = torch.zeros(max(self.n_edges, 1), dtype=torch.int64, device=d) if edges else None
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        check(lib().bfc_local_split(C.byref(self.g), split_wedges, ptr(cl), ptr(cr), ptr(ce),
                                    C.c_void_p(ws.data_ptr()), ws.numel(), _stream()),
              "local split")
        torch.cuda.synchronize(d)
        u = lambda t, n: t.cpu().numpy().view(np.uint64)[:n].copy() if t is not None else None
        return u(cl, self.n_left), u(cr, self.n_right), u(ce, self.n_edges)

    def local(self, vertices=True, edges=True):
        d = self.device
        cl = torch.zeros(max(self.n_left, 1), dtype=torch.int64, device=d) if vertices else None
        cr = torch.zeros(max(self.n_right, 1), dtype=torch.int64, device=d) if vertices else None
        ce = torch.zeros(max(self.n_edges, 1), dtype=torch.int64, device=d) if edges else None
        self.local_async(cl, cr, ce)
        torch.cuda.synchronize(d)
        u = lambda t, n: t.cpu().numpy().view(np.uint64)[:n].copy() if t is not None else None
        return u(cl, self.n_left), u(cr, self.n_right), u(ce, self.n_edges)

    # -------------------------------------------------------------- estimators
    def spar_buffers(self):
        """Workspace and outputs (beta, estimate, kept edges) for the sparsifier calls."""
        sz = C.c_size_t()
        check(lib().bfc_spar_ws_size(C.byref(self.g), C.byref(sz)), "spar ws size")
        return dict(ws=_bytes(sz.value, self.device),
                    out=torch.zeros(3, dtype=torch.int64, device=self.device))

    def _spar_async(self, fn, buf, param, seed, stream=None):
        ws, out = buf["ws"], buf["out"]
        check(fn(C.byref(self.g), param, seed, C.c_void_p(out.data_ptr()),
                 C.c_void_p(out.data_ptr() + 8), C.c_void_p(out.data_ptr() + 16),
                 C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "sparsifier")
        return buf

    def espar_async(self, buf, p, seed, stream=None):
        """Queue ESpar into buf["out"] = (beta, estimate bits, kept edges)."""
        return self._spar_async(lib().bfc_espar, buf, C.c_double(p), seed, stream)

    def clrspar_async(self, buf, ncolors, seed, stream=None):
        """Queue ClrSpar into buf["out"] = (beta, estimate bits, kept edges)."""
        return self._spar_async(lib().bfc_clrspar, buf, ncolors, seed, stream)

    @staticmethod
    def spar_result(buf):
        h = buf["out"].cpu().numpy()
        return int(h.view(np.uint64)[0]), float(h[1:2].view(np.float64)[0]), int(h.view(np.uint64)[2])

    def _spar(self, fn, param, seed):
        buf = self._spar_async(fn, self.spar_buffers(), param, seed)
        torch.cuda.synchronize(self.device)
        return self.spar_result(buf)

    def espar(self, p, seed):
        """ESpar: (kept butterflies, estimate, kept edges)."""
        return self._spar(lib().bfc_espar, C.c_double(p), seed)

    def clrspar(self, ncolors, seed):
        """ClrSpar: (monochromatic butterflies, estimate, kept edges)."""
        return self._spar(lib().bfc_clrspar, ncolors, seed)

    def check_probs(self, probs):
        """bfc_probs_check (synchronous): BfcError BFC_E_PROBS for invalid probabilities."""
        sz = C.c_size_t()
        check(lib().bfc_probs_check_ws_size(C.byref(sz)), "probs check ws size")
        ws = _bytes(sz.value, self.device)
        check(lib().bfc_probs_check(C.c_void_p(probs.data_ptr()), probs.numel(),
                                    C.c_void_p(ws.data_ptr()), ws.numel(), _stream()),
              "probabilities")

    def _samp(self, size_fn, fn, n, k, seed, probs, id_dtype):
        sz = C.c_size_t()
        check(size_fn(C.byref(self.g), k, C.byref(sz)), "sampler ws size")
        ws = _bytes(sz.value, self.device)
        ids = torch.zeros(max(k, 1), dtype=id_dtype, device=self.device)
        cnt = torch.zeros(max(k, 1), dtype=torch.int64, device=self.device)
        est = torch.zeros(1, dtype=torch.float64, device=self.device)
        pp = None
        if probs is not None:
            if isinstance(probs, torch.Tensor):
                pt = probs.to(device=self.device, dtype=torch.float64).contiguous()
            else:
                pt = torch.as_tensor(np.ascontiguousarray(probs, dtype=np.float64)).to(self.device)
            if pt.numel() != n:
                raise ValueError("probs has the wrong length")
            self.check_probs(pt)
            pp = C.c_void_p(pt.data_ptr())
        check(fn(C.byref(self.g), pp, k, seed, C.c_void_p(ids.data_ptr()),
                 C.c_void_p(cnt.data_ptr()), C.c_void_p(est.data_ptr()), C.c_void_p(ws.data_ptr()),
                 ws.numel(), _stream()), "sampler")
        torch.cuda.synchronize(self.device)
        ids_np = ids.cpu().numpy()
        ids_np = ids_np.view(np.uint32) if id_dtype == torch.int32 else ids_np.view(np.uint64)
        return ids_np[:k].copy(), cnt.cpu().numpy().view(np.uint64)[:k].copy(), float(est.item())

    def vsamp_buffers(self, k):
        """Device buffers for vsamp_async with k draws."""
        L = lib()
        sz = C.c_size_t()
        check(L.bfc_vsamp_ws_size(C.byref(self.g), k, C.byref(sz)), "vsamp ws size")
        return dict(ws=_bytes(sz.value, self.device), k=k,
                    ids=torch.zeros(max(k, 1), dtype=torch.int32, device=self.device),
                    cnt=torch.zeros(max(k, 1), dtype=torch.int64, device=self.device),
                    est=torch.zeros(1, dtype=torch.float64, device=self.device))

    def vsamp_async(self, buf, seed, probs=None, stream=None):
        """Queue VSamp with buf["k"] draws; probs a float64 device tensor or None."""
        ws = buf["ws"]
        check(lib().bfc_vsamp(C.byref(self.g),
                              C.c_void_p(probs.data_ptr()) if probs is not None else None,
                              buf["k"], seed, C.c_void_p(buf["ids"].data_ptr()),
                              C.c_void_p(buf["cnt"].data_ptr()), C.c_void_p(buf["est"].data_ptr()),
                              C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "vsamp")
        return buf["est"]

    def vsamp_draws_buffers(self, k):
        """Device buffers for vsamp_draws_async with k draws."""
        sz = C.c_size_t()
        check(lib().bfc_vsamp_draws_ws_size(C.byref(self.g), k, C.byref(sz)), "draws ws size")
        return dict(ws=_bytes(sz.value, self.device), k=k,
                    ids=torch.zeros(max(k, 1), dtype=torch.int32, device=self.device),
                    w=torch.zeros(max(k, 1), dtype=torch.int32, device=self.device),
                    total=torch.zeros(1, dtype=torch.int64, device=self.device))

    def vsamp_draws_async(self, buf, seed, probs=None, stream=None):
        """Queue VSamp's draws only (ids, integer weights, weight total)."""
        ws = buf["ws"]
        check(lib().bfc_vsamp_draws(C.byref(self.g),
                                    C.c_void_p(probs.data_ptr()) if probs is not None else None,
                                    buf["k"], seed, C.c_void_p(buf["ids"].data_ptr()),
                                    C.c_void_p(buf["w"].data_ptr()),
                                    C.c_void_p(buf["total"].data_ptr()),
                                    C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)),
              "vsamp draws")
        return buf

    def vsamp_draws(self, k, seed, probs=None):
        """VSamp's draws: (global ids, integer weights, weight total)."""
        if probs is not None:
            probs = torch.as_tensor(np.ascontiguousarray(probs, dtype=np.float64)
                                    if not isinstance(probs, torch.Tensor) else probs)
            probs = probs.to(device=self.device, dtype=torch.float64).contiguous()
        buf = self.vsamp_draws_async(self.vsamp_draws_buffers(k), seed, probs)
        torch.cuda.synchronize(self.device)
        return (buf["ids"].cpu().numpy().view(np.uint32)[:k].copy(),
                buf["w"].cpu().numpy().view(np.uint32)[:k].copy(),
                int(buf["total"].cpu().numpy().view(np.uint64)[0]))

    def vsamp(self, k, seed, probs=None):
        """VSamp: (drawn global ids, their counts, estimate)."""
        L = lib()
        return self._samp(L.bfc_vsamp_ws_size, L.bfc_vsamp, self.n_left + self.n_right, k, seed,
                          probs, torch.int32)

    def esamp(self, k, seed, probs=None):
        """ESamp: (drawn edge indices, their counts, estimate)."""
        L = lib()
        return self._samp(L.bfc_esamp_ws_size, L.bfc_esamp, self.n_edges, k, seed, probs,
                          torch.int64)

    def esamp_fast_buffers(self, k):
        """Device buffers for esamp_fast_async with k draws."""
        sz = C.c_size_t()
        check(lib().bfc_esamp_fast_ws_size(C.byref(self.g), k, C.byref(sz)), "esamp_fast ws size")
        return dict(ws=_bytes(sz.value, self.device), k=k,
                    eids=torch.zeros(max(k, 1), dtype=torch.int64, device=self.device),
                    hits=torch.zeros(max(k, 1), dtype=torch.int32, device=self.device),
                    est=torch.zeros(1, dtype=torch.float64, device=self.device))

    def esamp_fast_async(self, bufs, alpha, seed, probs=None, stream=None):
        """ESamp with Fast-eBFC into ``bufs`` (from esamp_fast_buffers), asynchronous;
        ``probs`` a device float64 tensor of n_edges, or None."""
        pp = None
        if probs is not None:
            if probs.numel() != self.n_edges or probs.dtype != torch.float64:
                raise ValueError("probs must be n_edges float64 values")
            pp = C.c_void_p(probs.data_ptr())
        ws = bufs["ws"]
        check(lib().bfc_esamp_fast(C.byref(self.g), pp, bufs["k"], alpha, seed,
                                   C.c_void_p(bufs["eids"].data_ptr()),
                                   C.c_void_p(bufs["hits"].data_ptr()),
                                   C.c_void_p(bufs["est"].data_ptr()), C.c_void_p(ws.data_ptr()),
                                   ws.numel(), _stream(stream)), "esamp_fast")

    def esamp_fast(self, k, alpha, seed, probs=None):
        """ESamp with Fast-eBFC: (drawn edge indices, hits per draw, estimate)."""
        bufs = self.esamp_fast_buffers(k)
        if probs is not None and not isinstance(probs, torch.Tensor):
            probs = torch.as_tensor(np.ascontiguousarray(probs, dtype=np.float64))
        if probs is not None:
            probs = probs.to(device=self.device, dtype=torch.float64).contiguous()
            self.check_probs(probs)
        self.esamp_fast_async(bufs, alpha, seed, probs)
        torch.cuda.synchronize(self.device)
        return (bufs["eids"].cpu().numpy().view(np.uint64)[:k].copy(),
                bufs["hits"].cpu().numpy().view(np.uint32)[:k].copy(),
                float(bufs["est"].item()))

    def wsamp_buffers(self, k):
        """Device buffers for wsamp_async with k draws."""
        sz = C.c_size_t()
        check(lib().bfc_wsamp_ws_size(C.byref(self.g), k, C.byref(sz)), "wsamp ws size")
        return dict(ws=_bytes(sz.value, self.device), k=k,
                    mids=torch.zeros(max(k, 1), dtype=torch.int32, device=self.device),
                    ends=torch.zeros(max(2 * k, 2), dtype=torch.int32, device=self.device),
                    cnt=torch.zeros(max(k, 1), dtype=torch.int64, device=self.device),
                    est=torch.zeros(1, dtype=torch.float64, device=self.device))

    def wsamp_async(self, bufs, seed, stream=None):
        """WSamp into ``bufs`` (from wsamp_buffers); no synchronisation."""
        ws = bufs["ws"]
        check(lib().bfc_wsamp(C.byref(self.g), bufs["k"], seed, C.c_void_p(bufs["mids"].data_ptr()),
                              C.c_void_p(bufs["ends"].data_ptr()),
                              C.c_void_p(bufs["cnt"].data_ptr()),
                              C.c_void_p(bufs["est"].data_ptr()), C.c_void_p(ws.data_ptr()),
                              ws.numel(), _stream(stream)), "wsamp")

    def wsamp(self, k, seed):
        """WSamp: (midpoints, ends (k, 2), counts, estimate); ids global (L, then n_left + R)."""
        bufs = self.wsamp_buffers(k)
        self.wsamp_async(bufs, seed)
        torch.cuda.synchronize(self.device)
        return (bufs["mids"].cpu().numpy().view(np.uint32)[:k].copy(),
                bufs["ends"].cpu().numpy().view(np.uint32)[:2 * k].reshape(k, 2).copy(),
                bufs["cnt"].cpu().numpy().view(np.uint64)[:k].copy(),
                float(bufs["est"].item()))

    def spar_eps_delta(self, kind, eps, delta, seed, B_pilot, log=None):
        """(eps, delta) estimate from ESpar or ClrSpar replicas (Sec. 6.1, 6.2): the lemma's
        rate from a pilot count and the largest degree, g groups of r replicas (replica i
        seeded seed + i) counted in one batch, the median of the group means.
        Returns (median, group means, p or N, g, r)."""
        kind_id = _lib.BFC_REPLICA_ESPAR if kind == "espar" else _lib.BFC_REPLICA_CLRSPAR
        p, nc = C.c_double(), C.c_uint32()
        check(lib().bfc_spar_threshold(kind_id, float(B_pilot),
                                       max(self.g.max_deg_l, self.g.max_deg_r),
                                       C.byref(p), C.byref(nc)), "threshold")
        g, r = C.c_uint32(), C.c_uint32()
        check(lib().bfc_eps_delta_plan(eps, delta, C.byref(g), C.byref(r)), "plan")
        g, r = g.value, r.value
        param = p.value if kind == "espar" else nc.value
        _, est, _ = self.spar_batch([(kind, param, seed + i) for i in range(g * r)], log=log)
        x = torch.as_tensor(np.ascontiguousarray(est, dtype=np.float64)).to(self.device)
        means = torch.zeros(g, dtype=torch.float64, device=self.device)
        med = torch.zeros(1, dtype=torch.float64, device=self.device)
        median_of_means(x, g, r, means, med)
        torch.cuda.synchronize(self.device)
        return float(med.item()), means.cpu().numpy(), param, g, r

    # -------------------------------------------------------------- batching
    def exact_tuned(self, tuning=None, side=BFC_SIDE_AUTO):
        """bfc_exact with a launch shape (a bfc_tuning, a dict of its fields, or None)."""
        t = _tuning(tuning)
        out = torch.zeros(1, dtype=torch.int64, device=self.device)
        ws = self.workspace(self.exact_ws_size(side))
        check(lib().bfc_exact_tuned(C.byref(self.g), side, C.byref(t) if t else None,
                                    C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()),
                                    ws.numel(), _stream()), "exact tuned")
        torch.cuda.synchronize(self.device)
        return int(out.cpu().numpy().view(np.uint64)[0])

    def autotune(self):
        """Fastest launch shape for this graph: (bfc_tuning, milliseconds)."""
        return _autotune(self, 0, None)

    def spar_batch(self, replicas, tuning=None, log=None):
        """Replicas [(kind, param, seed)] with kind "espar" (param p) or "clrspar" (param N),
        counted in one batch: (counts uint64[n], estimates float64[n], kept edges uint64[n]).
        ``log`` (optional) receives a line after each phase."""
        rb = ReplicaBatch(self, replicas, tuning=tuning, log=log)
        beta, est = rb.run()
        return beta, est, rb.kept

    def per_vertex(self):
        cl, cr, _ = self.local(vertices=True, edges=False)
        return cl, cr

    def per_edge(self):
        return self.local(vertices=False, edges=True)[2]


class ReplicaBatch:
    """ESpar / ClrSpar replicas of one graph counted together.

    Construction runs phase 1 (each replica's kept sizes; synchronous) and
    sizes the workspace; ``run_async`` queues phase 2 (kernels only, so it
    may be captured into a HIP graph and replayed) into device tensors.
    """

    def __init__(self, graph, replicas, tuning=None, log=None):
        L = lib()
        log = log or (lambda msg: None)
        self.graph = graph
        n = self.n = len(replicas)
        reps = self.reps = (_lib.bfc_replica * n)()
        for i, (kind, param, seed) in enumerate(replicas):
            if kind == "espar":
                reps[i] = _lib.bfc_replica(_lib.BFC_REPLICA_ESPAR, 0, float(param), seed)
            elif kind == "clrspar":
                reps[i] = _lib.bfc_replica(_lib.BFC_REPLICA_CLRSPAR, int(param), 0.0, seed)
            else:
                raise ValueError(kind)
        sz = C.c_size_t()
        g = C.byref(graph.g)
        check(L.bfc_spar_batch_filter_ws_size(g, n, C.byref(sz)), "filter ws size")
        ws = _bytes(sz.value, graph.device)
        info = self.info = (_lib.bfc_replica_info * n)()
        check(L.bfc_spar_batch_filter(g, n, reps, info, C.c_void_p(ws.data_ptr()), ws.numel(),
                                      _stream()), "batch filter")
        del ws
        check(L.bfc_spar_batch_ws_size(g, n, reps, info, C.byref(sz)), "batch ws size")
        self.ws_bytes = sz.value
        self.kept = np.array([info[i].kept for i in range(n)], dtype=np.uint64)
        starts = sum(info[i].n_right if info[i].sumsq_left < info[i].sumsq_right
                     else info[i].n_left for i in range(n))
        log(f"replica filter done: {int(self.kept.sum())} kept edges, "
            f"{starts} union start vertices, workspace {sz.value / 1e9:.1f} GB")
        self.ws = _bytes(sz.value, graph.device)
        self.tuning = _tuning(tuning)

    def run_async(self, beta, est, stream=None):
        """Queue phase 2: beta (int64) and est (float64) device tensors of n entries."""
        t = self.tuning
        check(lib().bfc_spar_batch(C.byref(self.graph.g), self.n, self.reps, self.info,
                                   C.byref(t) if t else None, C.c_void_p(beta.data_ptr()),
                                   C.c_void_p(est.data_ptr()), C.c_void_p(self.ws.data_ptr()),
                                   self.ws.numel(), _stream(stream)), "spar batch")

    def run(self):
        d = self.graph.device
        beta = torch.zeros(self.n, dtype=torch.int64, device=d)
        est = torch.zeros(self.n, dtype=torch.float64, device=d)
        self.run_async(beta, est)
        torch.cuda.synchronize(d)
        return beta.cpu().numpy().view(np.uint64).copy(), est.cpu().numpy().copy()


def median_of_means(x, groups, per_group, means, median, stream=None):
    """bfc_median_of_means on device float64 tensors (x: groups * per_group values)."""
    if x.numel() < groups * per_group or means.numel() < groups:
        raise ValueError("buffers too small")
    check(lib().bfc_median_of_means(C.c_void_p(x.data_ptr()), groups, per_group,
                                    C.c_void_p(means.data_ptr()), C.c_void_p(median.data_ptr()),
                                    _stream(stream)), "median of means")


def _tuning(t):
    if t is None:
        return None
    if isinstance(t, _lib.bfc_tuning):
        return t
    return _lib.bfc_tuning(**t)


def _autotune(graph, nparts, part_l):
    L = lib()
    sz = C.c_size_t()
    check(L.bfc_autotune_ws_size(C.byref(graph.g), C.byref(sz)), "autotune ws size")
    ws = _bytes(sz.value, graph.device)
    out = torch.zeros(max(nparts, 1), dtype=torch.int64, device=graph.device)
    best = _lib.bfc_tuning()
    ms = C.c_float()
    check(L.bfc_autotune(C.byref(graph.g), nparts,
                         C.c_void_p(part_l.data_ptr()) if part_l is not None else None,
                         C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                         _stream(), C.byref(best), C.byref(ms)), "autotune")
    return best, ms.value


class Batch:
    """Many bipartite graphs as one disjoint union, counted in one launch.

    ``graphs`` holds (n_left, n_right, l, r) tuples with ids local to each
    graph.  Each graph enters the union with its start side (ExactBFC's rule)
    as the union's L; ``swapped[q]`` tells whether its sides were exchanged.
    """

    def __init__(self, graphs, device="cuda"):
        L = lib()
        self.device = torch.device(device)
        ng = len(graphs)
        nl = np.array([g[0] for g in graphs], dtype=np.uint32)
        nr = np.array([g[1] for g in graphs], dtype=np.uint32)
        eoff = np.zeros(ng + 1, dtype=np.uint64)
        eoff[1:] = np.cumsum([len(g[2]) for g in graphs])
        l = np.concatenate([np.asarray(g[2], np.uint32) for g in graphs]) if ng else np.zeros(0)
        r = np.concatenate([np.asarray(g[3], np.uint32) for g in graphs]) if ng else np.zeros(0)
        dl = to_device_u32(l, self.device)
        dr = to_device_u32(r, self.device)
        m = int(eoff[-1])
        ul = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        ur = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        part_l = np.zeros(ng + 1, dtype=np.uint32)
        part_r = np.zeros(ng + 1, dtype=np.uint32)
        swapped = np.zeros(max(ng, 1), dtype=np.uint8)
        p32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_uint32))
        sz = C.c_size_t()
        check(L.bfc_batch_union_ws_size(ng, p32(nl), p32(nr),
                                        eoff.ctypes.data_as(C.POINTER(C.c_uint64)),
                                        C.byref(sz)), "union ws size")
        ws = _bytes(sz.value, self.device)
        check(L.bfc_batch_union(ng, p32(nl), p32(nr), eoff.ctypes.data_as(C.POINTER(C.c_uint64)),
                                C.c_void_p(dl.data_ptr()), C.c_void_p(dr.data_ptr()),
                                C.c_void_p(ul.data_ptr()), C.c_void_p(ur.data_ptr()),
                                p32(part_l), p32(part_r),
                                swapped.ctypes.data_as(C.POINTER(C.c_uint8)),
                                C.c_void_p(ws.data_ptr()), ws.numel(), _stream()), "batch union")
        del ws, dl, dr
        self.n_graphs = ng
        self.part_l_host, self.part_r_host = part_l, part_r
        self.swapped = swapped[:ng].astype(bool)
        self.part_l = to_device_u32(part_l, self.device)
        self.part_r = to_device_u32(part_r, self.device)
        self.graph = Graph(int(part_l[-1]), int(part_r[-1]), ul[:m], ur[:m], device=self.device,
                           parts=(self.part_l, self.part_r) if ng > 0 else None)
        del ul, ur
        check(L.bfc_exact_parts_ws_size(C.byref(self.graph.g), C.byref(sz)), "parts ws size")
        self.ws = _bytes(sz.value, self.device)

    @property
    def wedges(self):
        return self.graph.wedges(BFC_SIDE_L)

    def totals_async(self, out, tuning=None, stream=None):
        """Queue the per-graph counts into ``out`` (int64 device tensor, n_graphs)."""
        t = _tuning(tuning)
        check(lib().bfc_exact_parts(C.byref(self.graph.g), self.n_graphs,
                                    C.c_void_p(self.part_l.data_ptr()),
                                    C.byref(t) if t else None, C.c_void_p(out.data_ptr()),
                                    C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                    _stream(stream)), "exact parts")
        return out

    def totals(self, tuning=None):
        out = torch.zeros(max(self.n_graphs, 1), dtype=torch.int64, device=self.device)
        self.totals_async(out, tuning)
        torch.cuda.synchronize(self.device)
        return out.cpu().numpy().view(np.uint64)[:self.n_graphs].copy()

    def autotune(self):
        return _autotune(self.graph, self.n_graphs, self.part_l)


def exact(n_left, n_right, l, r, side=BFC_SIDE_AUTO):
    return Graph(n_left, n_right, l, r).exact(side)
