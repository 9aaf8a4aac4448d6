#!/usr/bin/env python3
"""Benchmark: exact butterfly counting on one MI355X.

One step is one pass of the hot path over the resident graph: ExactBFC's
per-call plan (segments at window boundaries, per-start wedge counts, work
queue), the exact count, and the per-vertex + per-edge counts.  The CSR build
happens once before the timed region and is reported separately.

value = wedges of the graph (sum over midpoints of C(d,2), the work of the
exact count) per second of step time.  The dominant-kernel roofline is for
the exact-count kernel, timed with HIP events on the stream it runs on.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
Z95 = 1.959963984540054
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1801_00338_amd", "csrc", "count.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload, kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def host_cpu():
    """CPU model and the cores this process may use (its affinity mask)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail, os.cpu_count() or 1


def _time_oracle_slice(w, l, r, side, target_s, threads):
    """ExactBFC of the oracle over the highest-id starts (the busiest ones in
    its id order), grown until the counting takes about target_s."""
    import oracle
    oracle.set_threads(threads)
    nA = w.nl if side == 1 else w.nr
    t0 = time.perf_counter()
    oracle.exact_range(w.nl, w.nr, l, r, side, 0, 0)
    t_build = time.perf_counter() - t0
    k = 2000 * threads
    while True:
        k = min(k, nA)
        t0 = time.perf_counter()
        _, wed, _ = oracle.exact_range(w.nl, w.nr, l, r, side, nA - k, nA)
        dt = time.perf_counter() - t0
        count_s = max(dt - t_build, 1e-9)
        if count_s >= target_s or k >= nA:
            break
        k = int(k * max(2.0, 1.5 * target_s / count_s))
    oracle.set_threads(1)
    return wed / count_s, (f"ExactBFC over the {k} highest-id starts of side "
                           f"{'L' if side == 1 else 'R'} ({wed} wedges, {count_s:.1f} s counting "
                           f"after a {t_build:.1f} s adjacency build), {threads} thread(s)")


def cpu_baseline(w, l, r, side, target_s):
    """The CPU oracle timed on this host on a bounded slice of start vertices:
    threads over starts on every core this process may use (at most 16, the
    host share of one GPU), and one thread for reference."""
    import oracle
    oracle.build(force=False)
    model, avail, nproc = host_cpu()
    threads = max(1, min(16, avail))
    v_all, s_all = _time_oracle_slice(w, l, r, side, target_s, threads)
    v_one, s_one = _time_oracle_slice(w, l, r, side, target_s / 2, 1)
    return {
        "value": v_all, "unit": "wedges/s", "cores": threads, "kind": "oracle",
        "sample": s_all, "cpu_model": model, "nproc": nproc, "cores_available": avail,
        "one_thread": {"value": v_one, "sample": s_one},
    }


def _sigma1(cnt, w=None):
    """Standard deviation of one VSamp draw's term B_v / (4 q_v) (q_v = w_v / sum w, or 1/n)."""
    import numpy as np
    c = cnt.astype(np.float64)
    B = c.sum() / 4
    if w is None:
        return math.sqrt(max(len(c) * np.dot(c, c) / 16 - B * B, 0.0))
    nz = c > 0
    q = w[nz] / w.sum()
    return math.sqrt(max(float(np.sum(c[nz] ** 2 / (16 * q))) - B * B, 0.0))


# budgets: the 1-2-5 grid from 1e3; the error check stops at 1e6 draws per query
GRID = [int(a * 10 ** e) for e in range(3, 9) for a in (1, 2, 5)]
KMAX_CHECK = 1_000_000


def vsamp_combine(counts, weights, total, k, n, weighted):
    """VSamp's estimate from per-draw counts in the library's order: weighted,
    count_i * (Q / (4 w_i)) summed left to right in blocks of 1,024 draws,
    the block sums left to right, over k; uniform, the exact integer sum
    times n / (4 k)."""
    import numpy as np
    if not weighted:
        return (float(int(counts.sum(dtype=np.uint64))) * float(n)) / (4.0 * float(k))
    t = counts.astype(np.float64) * (float(total) / (4.0 * weights.astype(np.float64)))
    parts = [np.cumsum(t[b:b + 1024])[-1] for b in range(0, k, 1024)]
    return float(np.cumsum(parts)[-1]) / float(k)


def learned_vs_uniform(dev, trials):
    """GPU time to 1% relative error at 95% confidence: learned importance vs uniform VSamp.

    Train the network on 16 Chung-Lu graphs (1M-20M edges, |L|:|R| = 1:4)
    from their exact per-vertex counts, then sample the 20M/80M/400M-edge
    graph.  For each method and each budget k of the 1-2-5 grid from 1,000
    (up to 1e6 draws), the 95th percentile of the relative error over
    `trials` seeds is measured against the exact count; the smallest budget
    at or below 1% is timed as one full query with HIP events (learned:
    features, inference and probabilities included).  The closed-form
    single-draw deviation is reported beside it as a cross-check.
    """
    import numpy as np
    import torch

    from paper_1801_00338_amd import api, gen, learned

    stream = torch.cuda.current_stream(dev)

    def events():
        return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    t0 = time.perf_counter()
    train = gen.training_graphs(16, 1_000_000, 20_000_000, seed=5)
    log(f"learned: generated 16 training graphs ({sum(len(t[2]) for t in train)} edges) "
        f"in {time.perf_counter() - t0:.1f} s")
    e0, e1 = events()
    e0.record(stream)
    x, t = learned.training_set(train, device=dev)
    e1.record(stream)
    torch.cuda.synchronize(dev)
    prep_ms = e0.elapsed_time(e1)
    del train
    net = learned.Mlp.init(7)
    steps = 3000
    orders = learned.Mlp.batch_orders(x.shape[0], steps, 65536, 1, dev)   # seeded inputs
    torch.cuda.synchronize(dev)
    e0, e1 = events()
    e0.record(stream)
    losses = net.train(x, t, steps=steps, batch=65536, lr=1e-3, seed=1, log_every=steps // 6,
                       orders=orders)
    e1.record(stream)
    torch.cuda.synchronize(dev)
    train_ms = e0.elapsed_time(e1)
    log(f"learned: {x.shape[0]} training rows, {steps} Adam steps in {train_ms:.0f} ms; "
        f"batch losses {[round(v, 4) for v in losses]}")
    del x, t, orders

    w5 = gen.WORKLOADS["chung_lu_20m_80m_400m"]
    t0 = time.perf_counter()
    l, r = w5.edges()
    log(f"learned: generated {w5.name} in {time.perf_counter() - t0:.1f} s")
    g = api.Graph(w5.nl, w5.nr, l, r, device=dev)
    del l, r
    B = g.exact()
    # the exact answers, timed for context: the exact count and the exact per-vertex counts
    tot = torch.zeros(1, dtype=torch.int64, device=dev)
    e0, e1 = events()
    e0.record(stream)
    g.exact_async(tot)
    e1.record(stream)
    e2, e3 = events()
    e2.record(stream)
    cnt = learned.vertex_counts(g)
    e3.record(stream)
    torch.cuda.synchronize(dev)
    exact_ms, vertex_ms = e0.elapsed_time(e1), e2.elapsed_time(e3)
    cnt_h = cnt.cpu().numpy().view(np.uint64)
    del cnt
    if int(cnt_h[:w5.nl].sum()) != 2 * B:
        raise SystemExit("per-vertex counts disagree with the exact count")
    log(f"learned: held-out graph B={B}")

    # the learned query's fixed part: features, inference, probabilities
    def query():
        return learned.learned_probs(g, net, floor_frac=0.05)
    query()
    qe = [events() for _ in range(3)]
    for a_, b_ in qe:
        a_.record(stream)
        probs = query()
        b_.record(stream)
    torch.cuda.synchronize(dev)
    query_ms = sorted(a_.elapsed_time(b_) for a_, b_ in qe)[1]
    p = probs.cpu().numpy()
    wq = np.where(p > 0, np.maximum(1.0, np.floor(p / p.max() * 4294967295.0)), 0.0)
    s_l = _sigma1(cnt_h, wq)
    s_u = _sigma1(cnt_h)
    n = w5.nl + w5.nr

    def timed(name, k, pr):
        buf = g.vsamp_buffers(k)
        g.vsamp_async(buf, 12345, pr)
        torch.cuda.synchronize(dev)
        ts = []
        for i in range(2):
            a_, b_ = events()
            a_.record(stream)
            g.vsamp_async(buf, 777 + i, pr)
            b_.record(stream)
            torch.cuda.synchronize(dev)
            ts.append(a_.elapsed_time(b_))
        log(f"learned: {name} query with k={k}: {min(ts):.1f} ms")
        return min(ts), buf

    def errors(name, pr, k):
        """Relative errors of `trials` seeded queries with k draws.  The
        draws come from the library (bfc_vsamp_draws: the same ids as
        bfc_vsamp for the same seed); each drawn vertex's count is read from
        the exact per-vertex counts in hand and the estimate formed in
        bfc_vsamp's order (checked bit for bit against bfc_vsamp below)."""
        buf = g.vsamp_draws_buffers(k)
        errs = []
        for t in range(trials):
            g.vsamp_draws_async(buf, (5 << 40) | t, pr)
            torch.cuda.synchronize(dev)
            ids = buf["ids"].cpu().numpy().view(np.uint32)[:k]
            w = buf["w"].cpu().numpy().view(np.uint32)[:k]
            Q = int(buf["total"].cpu().numpy().view(np.uint64)[0])
            e = vsamp_combine(cnt_h[ids], w, Q, k, n, pr is not None)
            errs.append(abs(e - B) / B)
        p95 = float(np.quantile(errs, 0.95))
        log(f"learned: {name}: k={k}: p95 rel. err over {trials} seeds {p95:.5f}")
        return p95

    out = {"workload": w5.describe(), "butterflies": B, "exact_count_ms": exact_ms,
           "exact_per_vertex_ms": vertex_ms, "train_graphs": 16,
           "train_rows_prep_ms": prep_ms, "train_ms": train_ms, "train_steps": steps,
           "floor_frac": 0.05,
           "method": (f"95th percentile of |Y - B| / B over {trials} seeds per budget on the "
                      "1-2-5 grid from 1,000 draws; the smallest budget at or below 1% is timed "
                      "as one full query")}
    res = {}
    for name, sig, pr in (("learned", s_l, probs), ("uniform", s_u, None)):
        d = {"sigma1": sig, "k_closed_form": math.ceil((Z95 * sig / (0.01 * B)) ** 2),
             "trials": trials, "p95_by_k": {}}
        reached = None
        for k in GRID:
            if k > KMAX_CHECK:
                break
            p95 = errors(name, pr, k)
            d["p95_by_k"][str(k)] = p95
            if p95 <= 0.01:
                reached = k
                break
        if reached is not None:
            ms, buf = timed(name, reached, pr)
            # the full query reproduces the estimate formed from the draws
            g.vsamp_async(buf, (5 << 40) | 0, pr)
            torch.cuda.synchronize(dev)
            ids = buf["ids"].cpu().numpy().view(np.uint32)[:reached]
            cnt_q = buf["cnt"].cpu().numpy().view(np.uint64)[:reached]
            if not np.array_equal(cnt_q, cnt_h[ids]):
                raise SystemExit("bfc_vsamp counts differ from the exact per-vertex counts")
            di, dw, dq = g.vsamp_draws(reached, (5 << 40) | 0, pr)
            e_host = vsamp_combine(cnt_h[di], dw, dq, reached, n, pr is not None)
            if not (np.array_equal(di, ids) and e_host == float(buf["est"].item())):
                raise SystemExit("bfc_vsamp's estimate differs from the one formed from its draws")
            d.update(reached=True, k=reached, p95_rel_err=d["p95_by_k"][str(reached)],
                     vsamp_ms=ms)
            del buf
        else:
            kk = max(int(x) for x in d["p95_by_k"])
            p95 = d["p95_by_k"][str(kk)]
            ms, buf = timed(name, kk, pr)
            del buf
            # the error falls as 1/sqrt(k): the budget 1% needs, from the measured p95
            k_need = math.ceil(kk * (p95 / 0.01) ** 2)
            d.update(reached=False, k_measured=kk, p95_at_k_measured=p95, ms_at_k_measured=ms,
                     k_needed_extrapolated=k_need,
                     note=(f"1% at 95% not reached by {kk} draws; the measured p95 at {kk} "
                           f"extrapolates (1/sqrt(k)) to {k_need} draws"))
            if k_need >= n:
                # more draws than vertices: the query then counts essentially every
                # vertex with a positive count, i.e. at least the exact per-vertex pass
                d["gpu_ms_to_1pct_lower_bound"] = max(vertex_ms, ms)
                d["note"] += ("; that exceeds n, so the query counts essentially every vertex: "
                              "its time is at least that of the exact per-vertex counts")
        if name == "learned":
            d["query_ms"] = query_ms
            d["gpu_ms_to_1pct"] = (query_ms + d["vsamp_ms"]) if d.get("reached") else None
        else:
            d["gpu_ms_to_1pct"] = d.get("vsamp_ms")
        res[name] = d
        log(f"learned: {name}: {d}")
    out.update(res)
    L_, U_ = res["learned"], res["uniform"]
    if L_.get("reached") and U_.get("reached"):
        out["speedup_vs_uniform"] = U_["gpu_ms_to_1pct"] / L_["gpu_ms_to_1pct"]
    elif L_.get("reached") and U_.get("gpu_ms_to_1pct_lower_bound"):
        out["speedup_vs_uniform_at_least"] = (U_["gpu_ms_to_1pct_lower_bound"] /
                                              L_["gpu_ms_to_1pct"])
    return out


def bench_batch(args):
    """Throughput of the batched exact count: 1,024 uneven graphs in one union."""
    import numpy as np
    import torch

    from paper_1801_00338_amd import api, gen

    t0 = time.perf_counter()
    graphs = gen.batch_graphs(1024, 1_000, 2_000_000, seed=3)
    m = sum(len(g[2]) for g in graphs)
    log(f"generated 1024 graphs, m={m} in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    b = api.Batch(graphs, device=dev)
    torch.cuda.synchronize(dev)
    build_ms = (time.perf_counter() - t0) * 1e3
    W = b.wedges
    best, tuned_ms = b.autotune()
    log(f"union built in {build_ms:.0f} ms; wedges={W}; autotuned {best.as_dict()} {tuned_ms:.2f} ms")
    out = torch.zeros(1024, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        b.totals_async(out, best)
    torch.cuda.synchronize(dev)
    ref = out.clone()
    # the timed step is one replay of the whole batched count captured in a HIP graph
    hg = capture(lambda: b.totals_async(out, best), dev)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        hg.replay()
        e1.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    if args.warmup and not torch.equal(out, ref):
        raise SystemExit("batch totals changed between runs")
    eager = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(3)]
    for e0, e1 in eager:
        e0.record(stream)
        b.totals_async(out, best)
        e1.record(stream)
    torch.cuda.synchronize(dev)
    ms = wall * 1e3 / args.steps
    line = {
        "metric": "graphs/s (batched exact counts)", "value": 1024 / (ms * 1e-3),
        "unit": "graphs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batch_1024 (m log-uniform in [1k, 2M], seed 3)", "graphs": 1024,
                   "edges": m, "wedges": W, "tuning": best.as_dict(),
                   "step": ("one replay of the HIP graph holding plan + exact count of every "
                            "graph + per-graph sums, one union")},
        "wedges_per_s": W / (ms * 1e-3),
        "gpu_ms_per_step": sum(e0.elapsed_time(e1) for e0, e1 in evs) / args.steps,
        "eager_gpu_ms": min(e0.elapsed_time(e1) for e0, e1 in eager),
        "union_build_once_ms": build_ms,
    }
    print(json.dumps(line), flush=True)


def bench_replicas(args):
    """The 256-replica ESpar/ClrSpar batch on the 10M/30M/100M-edge graph."""
    import numpy as np
    import torch

    from paper_1801_00338_amd import api, gen

    w = gen.WORKLOADS["chung_lu_10m_30m_100m"]
    l, r = w.edges()
    dev = torch.device("cuda:0")
    g = api.Graph(w.nl, w.nr, l, r, device=dev)
    del l, r
    B = g.exact()
    reps = []
    for p in (0.01, 0.02, 0.05, 0.1):
        reps += [("espar", p, (4 << 32) | len(reps) + i) for i in range(32)]
    for n in (4, 8, 16, 32):
        reps += [("clrspar", n, (4 << 32) | len(reps) + i) for i in range(32)]
    t0 = time.perf_counter()
    rb = api.ReplicaBatch(g, reps, log=log)
    phase1_ms = (time.perf_counter() - t0) * 1e3
    kept = rb.kept
    beta = torch.zeros(256, dtype=torch.int64, device=dev)
    est = torch.zeros(256, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    rb.run_async(beta, est)
    torch.cuda.synchronize(dev)
    ref_b, ref_e = beta.clone(), est.clone()
    # the timed step: one replay of phase 2 captured in a HIP graph
    hg = capture(lambda: rb.run_async(beta, est), dev)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(max(1, args.steps))]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        beta.fill_(-1)
        e0.record(stream)
        hg.replay()
        e1.record(stream)
        torch.cuda.synchronize(dev)
        if not (torch.equal(beta, ref_b) and torch.equal(est, ref_e)):
            raise SystemExit("a replay of the replica batch differs from the eager run")
    ms = min(e0.elapsed_time(e1) for e0, e1 in evs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    rb.run_async(beta, est)
    e1.record(stream)
    torch.cuda.synchronize(dev)
    eager_ms = e0.elapsed_time(e1)
    est = est.cpu().numpy()
    groups = {}
    for i in range(0, 256, 32):
        kind, param, _ = reps[i]
        e = est[i:i + 32]
        groups[f"{kind}:{param}"] = {"mean": float(e.mean()), "rel_err": float((e.mean() - B) / B),
                                     "var": float(e.var(ddof=1))}
    line = {
        "metric": "replicas/s (batched sparsification estimators)", "value": 256 / (ms * 1e-3),
        "unit": "replicas/s", "n_gpus": 1, "steps": len(evs), "warmup": 1,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": dict(w.describe(), replicas=256, butterflies=B, kept_edges=int(kept.sum()),
                       step=("one replay of the HIP graph holding phase 2: every replica's "
                             "keep flags, the union of the kept graphs, one count of all "
                             "replicas, the estimates")),
        "phase1_sizes_ms": phase1_ms, "eager_phase2_ms": eager_ms,
        "groups": groups,
    }
    print(json.dumps(line), flush=True)


def capture(fn, dev):
    """fn() captured once into a HIP graph (after one run outside the capture)."""
    import torch
    s = torch.cuda.Stream(dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream(dev).wait_stream(s)
    torch.cuda.synchronize(dev)
    hg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(hg):
        fn()
    torch.cuda.synchronize(dev)
    return hg


def bench_esamp_fast(args):
    """Time to 1% error at 95% confidence of ESamp with Fast-eBFC (Sec. 5.5) on one graph
    (default: the 1M/5M/50M-edge one), beside WSamp, ESamp with exact per-edge counts,
    uniform VSamp and the exact count.

    For each trial count alpha the variance of one draw's term is known in closed
    form from the exact per-edge counts: (m/4)^2 mean_e(B_e^2 + B_e (d_a d_x - B_e)
    / alpha) - B^2 (edge draw plus the binomial trials), which fixes the number of
    draws k; the fastest (k, alpha) is then checked over seeded queries.
    """
    import numpy as np
    import torch

    from paper_1801_00338_amd import api, gen

    w = gen.WORKLOADS[args.sampler_graph]
    t0 = time.perf_counter()
    l, r = w.edges()
    log(f"generated {w.name} in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    g = api.Graph(w.nl, w.nr, l, r, device=dev)
    m = l.size
    dd = (np.bincount(l, minlength=w.nl).astype(np.float64)[l] *
          np.bincount(r, minlength=w.nr).astype(np.float64)[r])
    del l, r
    B = g.exact()
    ts = []
    for _ in range(3):
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        g.exact()
        ts.append(time.perf_counter() - t0)
    exact_s = min(ts)
    ce = g.per_edge().astype(np.float64)
    log(f"B={B}, exact count {exact_s * 1e3:.1f} ms; per-edge counts read")
    assert abs(ce.sum() / 4 - B) < 1e-6 * B

    def k_for(v1):
        return int(math.ceil((Z95 * math.sqrt(max(v1, 0.0)) / (0.01 * B)) ** 2))

    def query_s(k, alpha, seeds=3):
        bufs = g.esamp_fast_buffers(k)
        g.esamp_fast_async(bufs, alpha, 1)
        torch.cuda.synchronize(dev)
        ts = []
        for s in range(seeds):
            t0 = time.perf_counter()
            g.esamp_fast_async(bufs, alpha, 2 + s)
            torch.cuda.synchronize(dev)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), bufs

    cands = []
    for alpha in (1, 4, 16, 64, 256, 1024):
        v1 = (m / 4) ** 2 * float(np.mean(ce * ce + ce * (dd - ce) / alpha)) - float(B) ** 2
        k = k_for(v1)
        if k >= 2**31:
            log(f"alpha={alpha}: k={k} too large")
            continue
        t, _ = query_s(k, alpha)
        log(f"alpha={alpha}: sigma1={math.sqrt(v1):.4g} k={k} query {t * 1e3:.2f} ms")
        cands.append((t, alpha, k, math.sqrt(v1)))
    t, alpha, k, sig = min(cands)

    def p95_of(run, budget_s):
        errs, t0 = [], time.perf_counter()
        for s in range(args.trials):
            if time.perf_counter() - t0 > budget_s:
                break
            errs.append(abs(run((5 << 40) | s) - B) / B)
        return float(np.percentile(errs, 95)), len(errs)

    def fast_run(bufs, seed):
        g.esamp_fast_async(bufs, alpha, seed)
        return float(bufs["est"].item())

    bufs = g.esamp_fast_buffers(k)
    p95, nseeds = p95_of(lambda sd: fast_run(bufs, sd), 60.0)
    log(f"best alpha={alpha} k={k}: {t * 1e3:.2f} ms; p95 error {p95:.4f} over {nseeds} seeds")
    k_closed = k
    if p95 > 0.01:
        # the closed form assumes a normal tail: grow k by the measured shortfall, once
        k = int(math.ceil(k * (p95 / 0.01) ** 2 * 1.05))
        del bufs
        t, bufs = query_s(k, alpha)
        p95, nseeds = p95_of(lambda sd: fast_run(bufs, sd), 60.0)
        log(f"resized k={k}: {t * 1e3:.2f} ms; p95 error {p95:.4f} over {nseeds} seeds")
    del bufs
    # ESamp with exact per-edge counts (Sec. 5.2) at its own k
    v1e = (m / 4) ** 2 * float(np.mean(ce * ce)) - float(B) ** 2
    ke = k_for(v1e)
    t0 = time.perf_counter()
    g.esamp(ke, 11)
    esamp_s = time.perf_counter() - t0
    log(f"ESamp with exact eBFC: k={ke}, {esamp_s * 1e3:.1f} ms")
    # WSamp (Sec. 5.3): sigma1 from a pilot of 4M draws, then the query at its k
    Wt = g.g.wedges_mid_l + g.g.wedges_mid_r
    pilot = g.wsamp_buffers(4_000_000)
    g.wsamp_async(pilot, 3)
    torch.cuda.synchronize(dev)
    sig_w = (Wt / 4) * float(pilot["cnt"].double().std())
    del pilot
    def wsamp_at(kw):
        bw = g.wsamp_buffers(kw)
        g.wsamp_async(bw, 4)
        torch.cuda.synchronize(dev)
        tw = []
        for s_ in range(3):
            t0 = time.perf_counter()
            g.wsamp_async(bw, 5 + s_)
            torch.cuda.synchronize(dev)
            tw.append(time.perf_counter() - t0)

        def run(seed):
            g.wsamp_async(bw, seed)
            return float(bw["est"].item())

        p, n = p95_of(run, 30.0)
        return float(np.median(tw)), p, n

    kw = k_for(sig_w ** 2)
    kw_closed = kw
    tw, p95w, nw = wsamp_at(kw)
    if p95w > 0.01:
        kw = int(math.ceil(kw * (p95w / 0.01) ** 2 * 1.05))
        tw, p95w, nw = wsamp_at(kw)
    wsamp = {"k": kw, "k_from_pilot": kw_closed, "s": tw, "sigma1_pilot": sig_w,
             "p95_rel_err": p95w, "seeds": nw}
    log(f"WSamp: {wsamp}")
    # VSamp (Sec. 5.1), uniform: closed-form k from the exact per-vertex counts
    cl, cr = g.per_vertex()
    cv = np.concatenate([cl, cr]).astype(np.float64)
    kv = k_for(cv.size * float(np.dot(cv, cv)) / 16 - float(B) ** 2)
    kvt = min(kv, 1_000_000)
    bv = g.vsamp_buffers(kvt)
    g.vsamp_async(bv, 1)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    g.vsamp_async(bv, 2)
    torch.cuda.synchronize(dev)
    vsamp = {"k": kv, "timed_k": kvt, "s_at_timed_k": time.perf_counter() - t0}
    del bv
    log(f"VSamp uniform: {vsamp}")
    line = {
        "metric": "seconds to 1% error at 95% (ESamp with Fast-eBFC)", "value": t, "unit": "s",
        "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": t * 1e3, "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "u32 hits, f64 estimate",
        "data": "synthetic",
        "config": dict(w.describe(), butterflies=B, alpha=alpha, k=k, k_closed_form=k_closed,
                       sigma1=sig, p95_rel_err=p95, seeds=nseeds,
                       step="edge draws, position map, alpha trials per draw, estimate"),
        "esamp_exact_ebfc": {"k": ke, "s": esamp_s},
        "wsamp": wsamp,
        "vsamp_uniform": vsamp,
        "exact_count_s": exact_s,
        "candidates": [{"alpha": a_, "k": k_, "s": t_} for t_, a_, k_, _ in cands],
    }
    print(json.dumps(line), flush=True)


SIDE_GRAPHS = [   # (|L|, |R|, gamma_L, gamma_R), 10M edges each, expected degrees capped at 100k
    (1_000_000, 5_000_000, 2.1, 2.3), (5_000_000, 1_000_000, 2.3, 2.1),
    (2_000_000, 2_000_000, 2.1, 2.8), (2_000_000, 2_000_000, 2.8, 2.1),
    (2_000_000, 2_000_000, 2.5, 2.5), (500_000, 10_000_000, 2.4, 2.4),
]


def bench_side_ablation(args):
    """Exact count from L, from R and by the paper's rule (Sec. 4: start from R iff
    sum_L d^2 < sum_R d^2) on synthetic graphs across skews and side ratios: the
    time follows the wedges of the chosen start side, and the rule picks the side
    with fewer of them."""
    import torch

    from paper_1801_00338_amd import api, gen
    from paper_1801_00338_amd._lib import BFC_SIDE_AUTO, BFC_SIDE_L, BFC_SIDE_R

    dev = torch.device("cuda:0")
    rows = []
    for j, (nl, nr, gl, gr) in enumerate(SIDE_GRAPHS):
        l, r = gen.chung_lu(nl, nr, 10_000_000, gl, gr, 100_000, seed=(7 << 32) | j)
        g = api.Graph(nl, nr, l, r, device=dev)
        del l, r
        out = torch.zeros(1, dtype=torch.int64, device=dev)
        row = {"n_left": nl, "n_right": nr, "gamma_left": gl, "gamma_right": gr,
               "sumsq_left": g.g.sumsq_l, "sumsq_right": g.g.sumsq_r,
               "auto_side": "R" if g.side_used(BFC_SIDE_AUTO) == BFC_SIDE_R else "L"}
        counts = set()
        for name, side in (("L", BFC_SIDE_L), ("R", BFC_SIDE_R), ("auto", BFC_SIDE_AUTO)):
            g.exact_async(out, side)
            torch.cuda.synchronize(dev)
            counts.add(int(out.item()))
            ts = []
            for _ in range(max(1, args.steps)):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                g.exact_async(out, side)
                e1.record()
                torch.cuda.synchronize(dev)
                ts.append(e0.elapsed_time(e1))
            row[f"ms_{name}"] = min(ts)
            if name != "auto":
                row[f"wedges_{name}"] = g.wedges(side)
        assert len(counts) == 1, "the count must not depend on the side"
        row["butterflies"] = counts.pop()
        row["auto_is_faster_side"] = row["ms_auto"] <= 1.05 * min(row["ms_L"], row["ms_R"])
        log(json.dumps(row))
        rows.append(row)
        del g
        torch.cuda.empty_cache()
    worst = max(max(r_["ms_L"], r_["ms_R"]) / r_["ms_auto"] for r_ in rows)
    line = {
        "metric": "slowdown of the wrong start side over the paper's side choice (max)",
        "value": worst, "unit": "x", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": sum(r_["ms_auto"] for r_ in rows), "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "side_ablation (6 Chung-Lu graphs of 10M edges)",
                   "graphs": rows},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chung_lu_1m_5m_50m")
    ap.add_argument("--sampler-graph", default="chung_lu_1m_5m_50m",
                    help="graph of --workload samplers")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--exact-only", action="store_true",
                    help="the step is the plan and the exact count only (no local counts)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-uniform sampling measurement")
    ap.add_argument("--trials", type=int, default=200,
                    help="seeds per budget for the learned-vs-uniform error check")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB three times (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the exact count "
              "of one graph is not sharded here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1801_00338_amd import api, gen

    if args.copy_probe:
        n = args.copy_probe << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {n} bytes three times")
        return

    if args.workload == "batch_1024":
        return bench_batch(args)
    if args.workload == "replicas_256":
        return bench_replicas(args)
    if args.workload == "side_ablation":
        return bench_side_ablation(args)
    if args.workload in ("esamp_fast", "samplers"):
        return bench_esamp_fast(args)
    if args.workload == "learned_vs_uniform":
        d = learned_vs_uniform(torch.device("cuda:0"), args.trials)
        ms = d["learned"].get("gpu_ms_to_1pct")
        print(json.dumps({
            "metric": "GPU time to 1% rel. err at 95%, learned importance VSamp",
            "value": ms, "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": ms, "higher_is_better": False, "scaling": "strong",
            "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": "chung_lu_20m_80m_400m learned vs uniform VSamp"},
            "learned_vs_uniform": d}), flush=True)
        return
    w = gen.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    l, r = w.edges()
    log(f"generated {w.name}: m={l.size} in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    g = api.Graph(w.nl, w.nr, l, r, device=dev)
    torch.cuda.synchronize(dev)
    build_ms = (time.perf_counter() - t0) * 1e3
    W = g.wedges()
    side = g.side_used()
    log(f"graph built in {build_ms:.0f} ms; side={'L' if side == 1 else 'R'} wedges={W}")

    total = torch.zeros(1, dtype=torch.int64, device=dev)
    n_out = (1, 1, 1) if args.exact_only else (w.nl, w.nr, w.m)
    cl = torch.zeros(n_out[0], dtype=torch.int64, device=dev)
    cr = torch.zeros(n_out[1], dtype=torch.int64, device=dev)
    ce = torch.zeros(n_out[2], dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)
    ws_bytes = g.exact_ws_size() if args.exact_only else max(g.exact_ws_size(), g.local_ws_size())
    g.workspace(ws_bytes)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        g.exact_plan()
        if ev is not None:
            ev[1].record(stream)
        g.exact_count(total)
        if ev is not None:
            ev[2].record(stream)
        if not args.exact_only:
            g.local_async(cl, cr, ce)
        if ev is not None:
            ev[3].record(stream)

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup} queued")
    torch.cuda.synchronize(dev)
    ref_total = int(total.cpu().numpy().view(np.uint64)[0])
    log(f"warmup done: butterflies={ref_total}")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    got_total = int(total.cpu().numpy().view(np.uint64)[0])
    if args.warmup == 0:
        ref_total = got_total
    if got_total != ref_total:
        raise SystemExit(f"count changed between runs: {ref_total} vs {got_total}")
    # consistency of the local counts with the total (Lemma 1 and four edges per butterfly)
    if not args.exact_only:
        s_l = int(cl.sum().item())
        s_r = int(cr.sum().item())
        s_e = int(ce.sum().item())
        if not (s_l == s_r == 2 * ref_total and s_e == 4 * ref_total):
            raise SystemExit(f"local counts inconsistent: {s_l} {s_r} {s_e} vs B={ref_total}")

    plan_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    exact_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    local_ms = sum(e[2].elapsed_time(e[3]) for e in evs) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    nA = w.nl if side == 1 else w.nr
    # algorithmic bytes of one exact-count launch: each wedge reads its end
    # point id (4 B); each (start, midpoint) pair reads the midpoint, its
    # position in the midpoint's list and the list end (12 B); each start
    # reads its row offset (4 B).
    alg_bytes = 4 * W + 12 * w.m + 4 * (nA + 1)
    achieved = alg_bytes / (exact_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles(w.name, "k_exact")
    # local counts, algorithmic bytes: the exact walk's bytes (4 W + 12 m +
    # 8 n offsets), a second pass over the same wedges to scatter the pair
    # terms (4 W) and the uint64 results of every vertex and edge (8 (n + m)),
    # n = |L| + |R|.  This design walks every end point w != u instead of the
    # filtered ones, and reads the final counts back, so it moves about twice
    # that (design_bytes).
    n_all = w.nl + w.nr
    alg_local = 8 * W + 12 * w.m + 8 * n_all + 8 * (n_all + w.m)
    design_local = 16 * W + 32 * w.m + 8 * n_all + 4 * (nA + 1)
    achieved_local = alg_local / (max(local_ms, 1e-6) * 1e-3) / 1e9
    line = {
        "metric": "wedges/s + HBM GB/s (exact); GPU time to 1% rel. err, learned vs uniform vsamp",
        "value": W / (ms_per_step * 1e-3),
        "unit": "wedges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": dict(w.describe(), side="L" if side == 1 else "R", wedges=W,
                       butterflies=ref_total,
                       step=("plan + exact count" if args.exact_only else
                             "plan + exact count + per-vertex and per-edge counts")),
        "breakdown_ms": {"plan": plan_ms, "exact_count": exact_ms, "local_counts": local_ms,
                         "graph_build_once": build_ms},
        "exact_wedges_per_s": W / (exact_ms * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ("k_exact_hash_small + k_exact_hash_mid + k_exact_narrow + "
                                "k_exact_wide (one exact count)"),
                     "alg_bytes_per_launch": alg_bytes},
        "roofline_local": {"bound": "hbm", "achieved": achieved_local, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved_local / HBM_PEAK_GBS,
                           "traffic": traffic_from_profiles(w.name, "k_local"),
                           "kernel": "k_local_narrow + k_local_wide + k_local_finish (+ plan)",
                           "alg_bytes_per_launch": alg_local,
                           "design_bytes_per_launch": design_local},
    }
    if args.exact_only:
        del line["roofline_local"]
        line["breakdown_ms"].pop("local_counts")
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        line["cpu_baseline"] = cpu_baseline(w, l, r, side, args.cpu_seconds)
    if not args.no_learned:
        del g, cl, cr, ce, total
        torch.cuda.empty_cache()
        try:
            line["learned_vs_uniform"] = learned_vs_uniform(dev, args.trials)
        except Exception as e:          # reported, never hidden: the exact line still stands
            line["learned_vs_uniform"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"learned part failed: {e}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
