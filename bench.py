#!/usr/bin/env python
"""Benchmark: exact k-clique counting on one MI355X.

Workload (one "step"): the power-law graph -- Chung-Lu, n = 1,000,000, mean
degree 32 (about 16M undirected edges), degree exponent 2.1, expected degrees
capped at w_max = sqrt(sum of weights) ~ 5657 (Chung-Lu's admissibility bound,
see the design notes for why the 20k cap is not used at k = 7 and 10) -- is
validated, oriented by degeneracy order on the GPU, and counted at k = 4, 7 and
10 without pivoting, edge-centric, through the C ABI.  Inputs are resident in
HBM before the timed region starts.

Output: ONE JSON line on stdout (everything else goes to stderr):
  value      = edges per second of the whole step: m / (step time), where a step
               orients the graph and counts it at every k
  per_k      = GPU count time (HIP events), edges/s = m / count time and the
               comparison with the oracle's stored counts, per k
  roofline   = the dominant traversal launch against the VALU bound:
               algorithmic int32 lane-ops = 2 x (bitset words of every node of
               the Fig. 2 tree under that launch's roots), divided by the
               launch's HIP-event duration
  cpu_baseline = the CPU oracle timed on a bounded root sample of the same graph,
               on all host cores and on one
  literal_wmax20000 = the same graph family with w_max = 20000 at k = 4
  small, batched, dense_core, served = the other configurations (see their
               functions), each checked against the oracle where it can be
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 int32 lanes per clock (4 SIMD x 16) x 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# sources of the lane-walk launches (kernel, launch set-up, shared device code)
LANE_SOURCES = ("kc_count.hip", "kc_count_impl.h", "kc_extract.h", "kc_internal.h", "kc_lane.hip", "kc_lane_impl.h")


def lane_sources_sha256():
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for name in LANE_SOURCES:
        h.update(name.encode())
        with open(os.path.join(here, "paper_2104_13209_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def golden_counts(name):
    """{k: c_k} from a stored oracle fixture under tests/golden/ (written by the
    scripts there, which call only the oracle), or {} when it is missing."""
    out = {}
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 3 and parts[0] in ("c", "g"):
                out[int(parts[1])] = int(parts[2])
    return out


def measured_traffic(k, width_list):
    """HBM bytes of one lane-walk launch (width list, k) from the committed
    FETCH_SIZE / WRITE_SIZE record, or None when there is none or the lane-walk
    sources changed since the counters were taken."""
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", "k_lane_powerlaw_k10_hbm_counters.md")) as fh:
            line = next(x for x in fh if x.startswith("traffic-record: "))
    except (OSError, StopIteration):
        return None
    rec = json.loads(line[len("traffic-record: "):])
    if rec.get("lane_sources_sha256") != lane_sources_sha256() or rec.get("k") != k:
        return None
    b = rec["bytes_per_launch_by_width_list"].get(str(width_list))
    return int(b) if b is not None else None


_CPU_DAG = None


def _cpu_chunk(task):
    import oracle
    k, roots = task
    return oracle.count(_CPU_DAG, k, False, oracle.EC, roots=roots)


def cpu_baseline(g, ks, frac, seed=0):
    """The oracle on a bounded sample of the same workload: full degeneracy
    orientation (single thread), then every k over a random fraction of the edge
    roots, scaled to all roots -- once with the sample split over the host's
    cores (fork pool, started before this process touches the GPU) and once on
    one core."""
    global _CPU_DAG
    import multiprocessing as mp
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    d = oracle.orient(g, oracle.DEGENERACY)
    t_orient = time.perf_counter() - t0
    _CPU_DAG = d
    rng = np.random.default_rng(seed)
    nsamp = max(1, int(d.m * frac))
    roots = np.sort(rng.choice(d.m, size=nsamp, replace=False))
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    chunks = [roots[i::4 * cores] for i in range(4 * cores)]
    per_k = {}
    total_all, total_one = t_orient, t_orient
    with mp.get_context("fork").Pool(cores) as pool:
        for k in ks:
            t0 = time.perf_counter()
            c_all = sum(pool.map(_cpu_chunk, [(k, ch) for ch in chunks], chunksize=1))
            dt_all = time.perf_counter() - t0
            t0 = time.perf_counter()
            c_one = oracle.count(d, k, False, oracle.EC, roots=roots)
            dt_one = time.perf_counter() - t0
            assert c_all == c_one
            per_k[str(k)] = {"sample_count": str(c_one), "sample_s_all_cores": round(dt_all, 3),
                             "sample_s_one_core": round(dt_one, 3),
                             "est_count_s_all_cores": round(dt_all * d.m / nsamp, 2),
                             "est_count_s_one_core": round(dt_one * d.m / nsamp, 2)}
            total_all += dt_all * d.m / nsamp
            total_one += dt_one * d.m / nsamp
        pool.close()
        pool.join()   # the workers end before this process touches the GPU
    return {
        "value": g.m / total_all,
        "unit": "edges/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "full degeneracy orientation (%.2f s, one core) + counts at k=%s over %d random edge roots "
                  "(%.2f%% of %d) split over %d processes, times scaled to all roots"
                  % (t_orient, ",".join(map(str, ks)), nsamp, 100.0 * nsamp / d.m, d.m, cores),
        "single_core": {"value": g.m / total_one, "unit": "edges/s", "cores": 1},
        "orient_s": round(t_orient, 3),
        "per_k": per_k,
    }


def bench_batched(kc, ngraphs, k, reps):
    """Batched form vs plain per-graph launches on the batched workload: graphs/s,
    per-graph counts compared exactly."""
    import numpy as np
    import torch
    import synth
    from paper_2104_13209_amd import autotune
    t0 = time.perf_counter()
    b = synth.batch(ngraphs, seed=4)
    log("batch: %d graphs, %d vertices, %d edges (%.1f s)" % (b.ngraphs, b.n, b.nnz // 2, time.perf_counter() - t0))
    bd = kc.batch_to_device(b)
    plan, report = autotune.tune(b, k)
    log("autotuned plan: %s" % report)
    bg = kc.BatchGraph(bd, k, plan)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(reps):
        bg.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    gpu_ms = e0.elapsed_time(e1) / reps
    batched = bg.counts()
    # plain: one kc_orient + kc_count per graph, each on its own device CSR
    dev = bd.row_ptr.device
    graphs = [kc.to_device(b.graph(g), dev) for g in range(b.ngraphs)]
    nmax = max(g.n for g in graphs)
    nnzmax = max(g.nnz for g in graphs)
    ows = torch.empty(kc.orient_workspace_bytes(nmax, nnzmax, kc.ORDER_DEGREE), dtype=torch.uint8, device=dev)
    dag = kc.Dag(nmax, nnzmax // 2, 0, -1, 0, torch.empty(nmax + 1, dtype=torch.int32, device=dev),
                 torch.empty(max(nnzmax // 2, 1), dtype=torch.int32, device=dev),
                 torch.empty(max(nnzmax // 2, 1), dtype=torch.int32, device=dev),
                 torch.empty(nmax, dtype=torch.int32, device=dev))
    probe = kc.Dag(nmax, nnzmax // 2, 1024, -1, 0, dag.row_ptr, dag.col, dag.src, dag.perm)
    cws = torch.empty(kc.count_workspace_bytes(probe, k, False), dtype=torch.uint8, device=dev)
    plain = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, g in enumerate(graphs):
        d = kc.orient(g, kc.ORDER_DEGREE, validate=False, ws=ows, out=dag)
        plain.append(kc.count(d, k, ws=cws))
        if (i + 1) % 2000 == 0:
            log("plain: %d graphs (%.1f s)" % (i + 1, time.perf_counter() - t0))
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    mism = sum(1 for x, y in zip(batched, plain) if x != y)
    fix = golden_counts("batch_counts_k5.txt") if (ngraphs == 10000 and k == 5) else {}
    matches = all(batched[i] == fix[i] for i in range(b.ngraphs)) if len(fix) == b.ngraphs else None
    return {
        "workload": "%d graphs, n log-uniform [50, 5000], ER / Chung-Lu(2.3, w_max = n - 1) 50/50, mean degree "
                    "U[8, 64], seed 4 (%d vertices, %d edges, max degree %d)"
                    % (b.ngraphs, b.n, b.nnz // 2, bd.max_degree),
        "matches_oracle": matches,
        "k": k,
        "graphs_per_s": b.ngraphs / wall,
        "ms_per_batch": round(wall * 1e3, 3),
        "gpu_ms_per_batch": round(gpu_ms, 3),
        "plain_graphs_per_s": b.ngraphs / plain_s,
        "plain_s": round(plain_s, 3),
        "speedup_vs_plain": round(plain_s / wall, 2),
        "mismatches_vs_plain": mism,
        "total_cliques": str(sum(batched)),
        "plan": report,
        "hipgraph": True,
    }


def bench_literal(kc, ks, reps):
    """The power-law graph with expected degrees capped at 20,000 as the
    configuration states (its saturated core has a few hundred vertices):
    orientation and counts at the given k, checked against the oracle's stored
    counts.  k = 7 is outside the time budget of a benchmark step here (see the
    design notes), so the default is k = 4."""
    import torch
    import synth
    g = synth.config_powerlaw(wmax=20000.0)
    dev = torch.device("cuda:0")
    csr = kc.to_device(g, dev)
    d = kc.orient(csr, kc.ORDER_DEGENERACY)
    ws = torch.empty(kc.count_workspace_bytes(d, max(ks), False, kc.SCHEME_EC), dtype=torch.uint8, device=dev)
    fix = golden_counts("powerlaw_wmax20000_counts.txt")
    out = {"workload": "chung_lu(n=1000000, mean_deg=32, gamma=2.1, wmax=20000, seed=2)", "n": g.n, "m": g.m,
           "d_max": d.d_max, "degeneracy": d.degeneracy, "order": "degeneracy", "scheme": "EC"}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        kc.orient(csr, kc.ORDER_DEGENERACY, out=d)
    e1.record()
    torch.cuda.synchronize()
    out["orient_ms"] = round(e0.elapsed_time(e1) / reps, 3)
    for k in ks:
        c = kc.count(d, k, scheme=kc.SCHEME_EC, ws=ws)
        ms = []
        for _ in range(reps):
            p = kc.Profile()
            c = kc.count(d, k, scheme=kc.SCHEME_EC, ws=ws, profile=p)
            ms.append(p.ms_total)
        t = sum(ms) / len(ms)
        out[str(k)] = {"count": str(c), "count_ms": round(t, 3), "edges_per_s": g.m / (t / 1e3),
                       "matches_oracle": (c == fix[k]) if k in fix else None}
        log("literal: k=%d count %d in %.1f ms" % (k, c, t))
    return out


def bench_small(kc, reps):
    """The small plain-method workload: latency of orientation and of the k = 4
    count (degree order, vertex roots), the count checked against the oracle.
    Its 4-clique count is tiny (about 0.7 expected), so the triangle count of
    the same graph is checked as well."""
    import torch
    import oracle
    import synth
    g = synth.config_small()
    dev = torch.device("cuda:0")
    csr = kc.to_device(g, dev)
    d = kc.orient(csr, kc.ORDER_DEGREE)
    c = kc.count(d, 4, scheme=kc.SCHEME_VC)
    torch.cuda.synchronize()
    t_or, t_ct = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        d = kc.orient(csr, kc.ORDER_DEGREE)
        t1 = time.perf_counter()
        c = kc.count(d, 4, scheme=kc.SCHEME_VC)
        t2 = time.perf_counter()
        t_or.append((t1 - t0) * 1e3)
        t_ct.append((t2 - t1) * 1e3)
    od = oracle.orient(g, oracle.DEGREE)
    want = oracle.count(od, 4, False, oracle.VC)
    c3 = kc.count(d, 3, scheme=kc.SCHEME_VC)
    want3 = oracle.count(od, 3, False, oracle.VC)
    return {"workload": "Erdos-Renyi G(2000, 0.01), seed 1; k = 4, degree order, vertex roots, non-pivot",
            "n": g.n, "m": g.m, "count": str(c), "triangles": str(c3),
            "matches_oracle": c == want and c3 == want3,
            "orient_ms_p50": round(sorted(t_or)[len(t_or) // 2], 3),
            "count_ms_p50": round(sorted(t_ct)[len(t_ct) // 2], 3),
            "note": "launch- and latency-bound: host wall time per call, inputs resident"}


def bench_densecore(kc, reps):
    """Pivot count-all (every k, 128-bit) on the dense-core workload, with the
    counts compared to the oracle's stored in tests/golden/."""
    import torch
    import synth
    t0 = time.perf_counter()
    g = synth.config_densecore()
    log("dense core: n=%d m=%d (%.1f s)" % (g.n, g.m, time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    d = kc.orient(kc.to_device(g, dev), kc.ORDER_DEGENERACY)
    out = {"workload": "Chung-Lu background n=%d, mean degree 40, exponent 2.1, w_max 1000, seed 3, plus 50 "
                       "communities of U[60, 80] vertices at density 0.9; degeneracy order, pivoting, all k" % g.n,
           "n": g.n, "m": g.m, "d_max": d.d_max, "degeneracy": d.degeneracy}
    fixture = {}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "densecore_count_all.txt")
    if os.path.exists(path):
        with open(path) as f:
            for line in f:
                parts = line.split()
                if len(parts) == 3 and parts[0] == "c":
                    fixture[int(parts[1])] = int(parts[2])
    for name, scheme in (("vc", kc.SCHEME_VC), ("ec", kc.SCHEME_EC)):
        ws = torch.empty(kc.count_workspace_bytes(d, 0, True, scheme), dtype=torch.uint8, device=dev)
        got, omega = kc.count_all(d, pivot=True, scheme=scheme, ws=ws)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        profs = []
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            p = kc.Profile()
            got, omega = kc.count_all(d, pivot=True, scheme=scheme, ws=ws, profile=p)
            profs.append(p)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        # pivot roofline: the launch (light |S| <= 64 / heavy roots) with the
        # most time, its words read per node (|I| + 1 scoring rows + the child's
        # row) from an untimed stats pass, 2 int32 ops per word
        sp = kc.Profile()
        kc.count_all(d, pivot=True, scheme=scheme, ws=ws, profile=sp, collect_stats=True)
        launch_ms = [sum(p.ms_light for p in profs) / reps, sum(p.ms_heavy for p in profs) / reps]
        j = 0 if launch_ms[0] >= launch_ms[1] else 1
        achieved = 2.0 * sp.word_ops[j] / (launch_ms[j] / 1e3) / 1e12
        out[name] = {"count_all_ms": round(ms, 3), "edges_per_s": g.m / (ms / 1e3), "omega": omega,
                     "matches_oracle_counts": (got[:omega + 1] == [fixture.get(k) for k in range(omega + 1)])
                     if fixture else None,
                     "launch_ms": [round(x, 3) for x in launch_ms],
                     "roofline": {"bound": "alu", "kernel": "k_piv (%s roots, count-all)" % ("light", "heavy")[j],
                                  "achieved": round(achieved, 4), "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s",
                                  "frac": round(achieved / VALU_PEAK_TOPS, 5),
                                  "work": "2 int32 ops per bitset word: %d tree nodes reading %d words (scoring "
                                          "|I| + 1 rows per node, W words per child) in %.3f ms"
                                          % (sp.nodes[j], sp.word_ops[j], launch_ms[j])}}
        log("dense core %s: count-all %.1f ms, omega %d" % (name, ms, omega))
    out["total_cliques"] = str(sum(got[1:]))
    return out


def served_pool(ngraphs, nmin, nmax, seed=5):
    """Pool of graphs for serving: shapes uniform over {power-law Chung-Lu
    (gamma 2.1, mean 32, w_max = sqrt(sum w)), dense core (Chung-Lu background +
    planted communities of 20-60 at density 0.8), Erdos-Renyi / Chung-Lu(2.3) with
    mean degree U[8, 64]}, vertex counts log-uniform on [nmin, nmax]."""
    import synth
    graphs, kinds = [], []
    for i in range(ngraphs):
        u = synth.uniform(seed, 3 * i)
        n = int(math.exp(math.log(nmin) + u * (math.log(nmax) - math.log(nmin))))
        kind = int(synth.uniform(seed, 3 * i + 1) * 3)
        gs = seed * 100003 + i
        if kind == 0:
            g = synth.chung_lu(n, 2.1, 32.0, math.sqrt(32.0 * n), gs)
        elif kind == 1:
            g = synth.dense_core(n, 10.0, 2.1, max(1, n // 5000), 20, 60, 0.8, gs)
        else:
            d = 8.0 + 56.0 * synth.uniform(seed, 3 * i + 2)
            if synth.uniform(seed, 3 * i + 2 + 7919) < 0.5:
                g = synth.erdos_renyi(n, d / (n - 1), gs)
            else:
                g = synth.chung_lu(n, 2.3, d, math.sqrt(d * n), gs)
        graphs.append(g)
        kinds.append(kind)
        if (i + 1) % 25 == 0:
            log("served pool: %d of %d graphs generated" % (i + 1, ngraphs))
    return graphs, kinds


def percentile(xs, q):
    ys = sorted(xs)
    if not ys:
        return None
    i = min(len(ys) - 1, max(0, int(math.ceil(q / 100.0 * len(ys))) - 1))
    return ys[i]


def bench_served(kc, ngraphs, nmin, nmax, nq, nwarm, slots, budget_gb, util, seed=5):
    """Continuous batching (kc_server, `slots` workers) vs sequential launches
    (one worker) on the same Poisson trace of (graph, k, pivot) queries."""
    import numpy as np
    t0 = time.perf_counter()
    graphs, kinds = served_pool(ngraphs, nmin, nmax, seed)
    log("served pool: %d graphs, %d edges (%.1f s)" % (len(graphs), sum(g.m for g in graphs), time.perf_counter() - t0))
    dags = [kc.orient(kc.to_device(g), kc.ORDER_DEGENERACY, validate=False) for g in graphs]
    rng = np.random.default_rng(seed)
    total = nwarm + nq
    qs = [(int(rng.integers(0, ngraphs)), int(rng.integers(3, 13)), bool(rng.random() < 0.3)) for _ in range(total)]
    budget = int(budget_gb * (1 << 30))
    # service rate of sequential launches, measured back to back on the warm-up queries
    with kc.Server(dags, slots=1, mem_budget=budget) as sv:
        t0 = time.perf_counter()
        res = kc.replay_trace(sv, [(0.0, g, k, p) for g, k, p in qs[:nwarm]],
                              progress=lambda c: log("served: %d warm-up results" % c))
        seq_rate = nwarm / (time.perf_counter() - t0)
    log("served: sequential service rate %.1f queries/s" % seq_rate)
    lam = util * seq_rate
    gaps = rng.exponential(1.0 / lam, size=nq)
    arr = np.cumsum(gaps) - gaps[0]
    trace = [(float(a), g, k, p) for a, (g, k, p) in zip(arr, qs[nwarm:])]
    out = {}
    sweep = {}
    results = {}
    # the process has 4 hardware queues: slot counts around and above that
    for name, nslots in (("served", slots), ("sequential", 1), ("slots_2", 2), ("slots_4", 4)):
        if name.startswith("slots_") and nslots == slots:
            continue
        log("served: %s pass (%d slots, about %.0f s of arrivals) ..." % (name, nslots, trace[-1][0]))
        with kc.Server(dags, slots=nslots, mem_budget=budget) as sv:
            t0 = time.perf_counter()
            rs = kc.replay_trace(sv, trace, progress=lambda c: log("served: %d results" % c))
            span = max(r.t_done for r in rs) - min(r.t_submit for r in rs)
        lat = [r.latency * 1e3 for r in rs]
        log("served: %s pass done (%.1f s)" % (name, span))
        rec = {"slots": nslots, "queries_per_s": len(rs) / span, "p50_ms": round(percentile(lat, 50), 3),
               "p99_ms": round(percentile(lat, 99), 3), "mean_ms": round(sum(lat) / len(lat), 3),
               "refused": sum(1 for r in rs if r.status == kc.ENOMEM),
               "errors": sum(1 for r in rs if r.status not in (kc.OK, kc.ENOMEM))}
        sweep[str(nslots)] = rec
        if not name.startswith("slots_"):
            out[name] = rec
        results[nslots] = [(r.status, r.value) for r in rs]
    same = all(v == results[1] for v in results.values())
    out["slots_sweep"] = sweep
    # saturation: every query submitted at once (closed loop), throughput only
    for name, nslots in (("served_saturated", slots), ("sequential_saturated", 1)):
        with kc.Server(dags, slots=nslots, mem_budget=budget) as sv:
            rs = kc.replay_trace(sv, [(0.0, g, k, p) for _, g, k, p in trace],
                                 progress=lambda c: log("served: %d results" % c))
            span = max(r.t_done for r in rs) - min(r.t_submit for r in rs)
        log("served: %s pass done (%.1f s)" % (name, span))
        out[name] = {"queries_per_s": len(rs) / span}
    out.update({
        "workload": "%d graphs (n log-uniform [%d, %d], shapes power-law / dense-core / batch-like), %d queries "
                    "after %d warm-up, k U{3..12}, pivot p=0.3, Poisson arrivals at %.2f x the sequential service rate"
                    % (ngraphs, nmin, nmax, nq, nwarm, util),
        "arrival_rate_qps": lam,
        "sequential_service_qps": seq_rate,
        "memory_budget_bytes": budget,
        "results_identical": same,
    })
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ks", default="4,7,10")
    ap.add_argument("--wmax", type=float, default=0.0, help="0 = sqrt(sum w)")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--width", type=int, default=0)
    ap.add_argument("--scheme", type=int, default=2)
    ap.add_argument("--no-handoff", action="store_true", help="keep subtrees on the wavefront that found them")
    ap.add_argument("--cpu-frac", type=float, default=0.005)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-literal", action="store_true", help="skip the w_max = 20000 leg")
    ap.add_argument("--literal-ks", default="4", help="k of the w_max = 20000 leg")
    ap.add_argument("--batch-graphs", type=int, default=10000)
    ap.add_argument("--batch-k", type=int, default=5)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--serve-graphs", type=int, default=200)
    ap.add_argument("--serve-nmin", type=int, default=10000)
    ap.add_argument("--serve-nmax", type=int, default=100000)
    ap.add_argument("--serve-queries", type=int, default=600)
    ap.add_argument("--serve-warmup", type=int, default=60)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-util", type=float, default=0.7)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--dense-reps", type=int, default=2)
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this many MiB first (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): the counting path runs on a single MI355X; "
              "sharding over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2104_13209_amd as kc
    import synth

    ks = [int(x) for x in args.ks.split(",")]
    mean = 32.0
    wmax = args.wmax if args.wmax > 0 else math.sqrt(args.n * mean)
    t0 = time.perf_counter()
    g = synth.config_powerlaw(n=args.n, wmax=wmax)
    log("graph: n=%d m=%d max_deg=%d (%.1f s)" % (g.n, g.m, int(g.degrees().max()), time.perf_counter() - t0))

    cpu = None
    if not args.no_cpu:
        # before this process touches the GPU: the baseline forks worker processes
        log("cpu baseline (oracle, sampled) ...")
        t0 = time.perf_counter()
        cpu = cpu_baseline(g, ks, args.cpu_frac)
        log("cpu baseline took %.1f s" % (time.perf_counter() - t0))

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe_mib > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings give
        # the scale of the counters for the kernels that follow
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 3 x %d bytes" % nb)
        del src, dst
    csr = kc.to_device(g, dev)
    m = g.m
    order = kc.ORDER_DEGENERACY
    ows = torch.empty(kc.orient_workspace_bytes(g.n, g.nnz, order), dtype=torch.uint8, device=dev)
    dag = kc.Dag(g.n, m, 0, -1, order,
                 torch.empty(g.n + 1, dtype=torch.int32, device=dev),
                 torch.empty(m, dtype=torch.int32, device=dev),
                 torch.empty(m, dtype=torch.int32, device=dev),
                 torch.empty(g.n, dtype=torch.int32, device=dev))
    kc.orient(csr, order, validate=True, ws=ows, out=dag)
    cws = torch.empty(kc.count_workspace_bytes(dag, max(ks), False, args.scheme), dtype=torch.uint8, device=dev)
    log("dag: d_max=%d degeneracy=%d" % (dag.d_max, dag.degeneracy))

    orient_ms = []

    def step(profiles):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        kc.orient(csr, order, validate=True, ws=ows, out=dag)
        e1.record()
        e1.synchronize()
        if profiles is not None:
            orient_ms.append(e0.elapsed_time(e1))
        out = {}
        for k in ks:
            p = kc.Profile()
            out[k] = kc.count(dag, k, scheme=args.scheme, width=args.width, ws=cws, profile=p,
                              handoff=not args.no_handoff)
            if profiles is not None:
                profiles.setdefault(k, []).append(p)
        return out

    for i in range(args.warmup):
        t0 = time.perf_counter()
        counts = step(None)
        log("warmup %d: %.3f s counts=%s" % (i, time.perf_counter() - t0, counts))

    profiles = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        counts = step(profiles)
        log("step %d done (%.3f s elapsed)" % (i, time.perf_counter() - t0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps

    # the oracle's counts of this graph (tests/golden/powerlaw_counts.txt) when
    # the workload is the default one
    fix = golden_counts("powerlaw_counts.txt") if (args.n == 1_000_000 and args.wmax <= 0) else {}
    per_k = {}
    phases = []
    for k in ks:
        ps = profiles[k]
        ms = sum(p.ms_total for p in ps) / len(ps)
        ml = sum(p.ms_light for p in ps) / len(ps)
        mh = sum(p.ms_heavy for p in ps) / len(ps)
        mw = [sum(p.ms_width[j] for p in ps) / len(ps) for j in range(6)]
        per_k[str(k)] = {"count": str(counts[k]), "count_ms": round(ms, 3), "edges_per_s": m / (ms / 1e3),
                         "classify_ms": round(sum(p.ms_classify for p in ps) / len(ps), 3),
                         "light_ms": round(ml, 3), "heavy_ms": round(mh, 3),
                         "width_list_ms": [round(x, 3) for x in mw],
                         "width_list_roots": [int(ps[0].roots_width[j]) for j in range(6)],
                         "width_list_handoffs": [int(ps[-1].items_width[j]) for j in range(6)],
                         "matches_oracle": (counts[k] == fix[k]) if k in fix else None}
        phases.append((ms, k, mw))

    # dominant kernel launch: at the k that takes longest, the width-list launch
    # with the most wavefront time (launch span x busy fraction; the widest list
    # runs beside the others, so its span alone overstates it), and its
    # algorithmic work, from a separate, untimed stats pass of the same call
    _, dom_k, dom_mw = max(phases)
    sp = kc.Profile()
    c_stats = kc.count(dag, dom_k, scheme=args.scheme, width=args.width, ws=cws, profile=sp, collect_stats=True,
                       handoff=not args.no_handoff)
    assert c_stats == counts[dom_k]
    dom_j = max(range(6), key=lambda j: dom_mw[j] * float(sp.busy_width[j]))
    dom_ms = dom_mw[dom_j]
    # algorithmic work of that launch: the tree of Fig. 2 has one node per
    # l-clique for l = 3 .. k-1 under each edge root, each an AND + popcount over
    # the root's W words; untimed stats passes at k' = 3 .. k-1 give, per width
    # list, the k'-cliques weighted by their root's W (no pruning involved)
    alg_words = 0
    for kk in range(3, dom_k):
        cp = kc.Profile()
        kc.count(dag, kk, scheme=args.scheme, width=args.width, ws=cws, profile=cp, collect_stats=True,
                 handoff=not args.no_handoff)
        alg_words += int(cp.cwords_width[dom_j])
    achieved = 2.0 * alg_words / (dom_ms / 1e3) / 1e12
    achieved_expanded = 2.0 * sp.words_width[dom_j] / (dom_ms / 1e3) / 1e12
    roofline = {
        "bound": "alu",
        "kernel": "k_lane<MAXW=%d, %s> (width list %d, k=%d)" % (1 << dom_j, "EC" if args.scheme == 2 else "VC",
                                                               dom_j, dom_k),
        "achieved": round(achieved, 4),
        "peak": round(VALU_PEAK_TOPS, 2),
        "unit": "TOP/s",
        "frac": round(achieved / VALU_PEAK_TOPS, 5),
        "traffic": measured_traffic(dom_k, dom_j),
        "traffic_source": "FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (copy-calibrated) for this launch; profiles/k_lane_powerlaw_k10_hbm_counters.md",
        "work": "2 int32 ops (AND + popcount) per bitset word per node of the Fig. 2 tree (one node per "
                "l-clique, l = 3..%d, W = the root's words): %d words in one launch of %.3f ms (HIP events, "
                "mean of timed steps)" % (dom_k - 1, alg_words, dom_ms),
        "expanded": {"nodes": int(sp.nodes_width[dom_j]), "words": int(sp.words_width[dom_j]),
                     "achieved": round(achieved_expanded, 4),
                     "frac": round(achieved_expanded / VALU_PEAK_TOPS, 5),
                     "note": "nodes the kernel expands after size pruning (sets too small to complete a "
                             "k-clique are skipped), leaf level counted as edge counts"},
        "lane_expansions_per_round": round(sp.expand_width[dom_j] / max(1, 64 * sp.iters_width[dom_j]), 4),
        "wavefront_busy_fraction": round(float(sp.busy_width[dom_j]), 4),
        "wavefronts": int(sp.waves_width[dom_j]),
        "width_list_busy_fraction": [round(float(sp.busy_width[j]), 4) for j in range(6)],
        "width_list_nodes": [int(sp.nodes_width[j]) for j in range(6)],
        "width_list_wave_iterations": [int(sp.iters_width[j]) for j in range(6)],
        "width_list_expansions": [int(sp.expand_width[j]) for j in range(6)],
    }

    # ablation (Sec. 4.3): the same counts without binary encoding, at small k
    ablation = {"workload": "the timed graph, edge roots", "note": "KC_OPT_NO_BITSETS: sorted candidate lists, "
                "binary-search intersections in the oriented CSR, one wavefront per root"}
    for k in (4, 5):
        pb, pl = kc.Profile(), kc.Profile()
        cb = kc.count(dag, k, scheme=kc.SCHEME_EC, ws=cws, profile=pb)
        cl = kc.count(dag, k, scheme=kc.SCHEME_EC, ws=cws, profile=pl, bitsets=False)
        ablation[str(k)] = {"bitsets_ms": round(pb.ms_total, 3), "lists_ms": round(pl.ms_total, 3),
                            "bitset_speedup": round(pl.ms_total / pb.ms_total, 2), "same_count": cb == cl}
    log("ablation: %s" % ablation)

    # orientation criteria (Sec. 3.1, Table 2's trade-off): orientation time, the
    # DAG's out-degree bound and the count at k = 4 and 7 under each order (k = 4
    # only for the colouring order: its hubs keep thousands of out-neighbours, so
    # deep counts take minutes there)
    orders = {}
    for name, oc in (("degree", kc.ORDER_DEGREE), ("degeneracy", kc.ORDER_DEGENERACY),
                     ("approx_degeneracy", kc.ORDER_APPROX_DEGENERACY), ("colour", kc.ORDER_COLOR)):
        ows_or = torch.empty(kc.orient_workspace_bytes(g.n, g.nnz, oc), dtype=torch.uint8, device=dev)
        od = kc.orient(csr, oc, validate=False, ws=ows_or)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            kc.orient(csr, oc, validate=False, ws=ows_or, out=od)
        e1.record()
        e1.synchronize()
        ent = {"orient_ms_no_validation": round(e0.elapsed_time(e1) / args.steps, 3), "d_max": od.d_max}
        del ows_or
        ows_o = torch.empty(kc.count_workspace_bytes(od, 7, False, kc.SCHEME_EC), dtype=torch.uint8, device=dev)
        for k in ((4,) if oc == kc.ORDER_COLOR else (4, 7)):
            p = kc.Profile()
            c = kc.count(od, k, scheme=kc.SCHEME_EC, ws=ows_o, profile=p)
            ent[str(k)] = {"count_ms": round(p.ms_total, 3), "matches_oracle": (c == fix[k]) if k in fix else None}
        orders[name] = ent
        del ows_o
        log("order %s: %s" % (name, ent))

    # listing (kc_list): every triangle of the timed graph, 3 input ids per row
    listing = None
    if 3 in fix or args.n == 1_000_000:
        c3 = kc.count(dag, 3, scheme=kc.SCHEME_EC, ws=cws)
        rows_ws = torch.empty(kc.count_workspace_bytes(dag, 3, False, kc.SCHEME_EC), dtype=torch.uint8, device=dev)
        kc.list_cliques(dag, 3, cap=c3, scheme=kc.SCHEME_EC, ws=rows_ws)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        total, rows = kc.list_cliques(dag, 3, cap=c3, scheme=kc.SCHEME_EC, ws=rows_ws)
        e1.record()
        e1.synchronize()
        ms_l = e0.elapsed_time(e1)
        listing = {"k": 3, "rows": int(total), "list_ms": round(ms_l, 3), "rows_per_s": total / (ms_l / 1e3),
                   "output_GB_per_s": round(12.0 * total / (ms_l / 1e3) / 1e9, 2),
                   "matches_oracle": (total == fix[3]) if 3 in fix else None}
        del rows, rows_ws
        log("listing: %s" % listing)

    literal = None
    if not args.no_literal and args.n == 1_000_000:
        log("literal w_max = 20000 leg ...")
        literal = bench_literal(kc, [int(x) for x in args.literal_ks.split(",")], args.steps)

    batched = None
    if not args.no_batch:
        log("batched form ...")
        batched = bench_batched(kc, args.batch_graphs, args.batch_k, args.batch_reps)
        log("batched: %.0f graphs/s vs plain %.0f graphs/s" % (batched["graphs_per_s"], batched["plain_graphs_per_s"]))

    small = bench_small(kc, 20)
    log("small: orient %.3f ms, count %.3f ms" % (small["orient_ms_p50"], small["count_ms_p50"]))

    dense = None
    if not args.no_dense:
        log("dense-core form ...")
        dense = bench_densecore(kc, args.dense_reps)

    served = None
    if not args.no_serve:
        log("served form ...")
        served = bench_served(kc, args.serve_graphs, args.serve_nmin, args.serve_nmax, args.serve_queries,
                              args.serve_warmup, args.serve_slots, args.serve_budget_gb, args.serve_util)
        log("served: %s" % {k: v for k, v in served.items() if k in ("served", "sequential")})

    res = {
        "metric": "count time + edges/s at k=4,7,10 (non-pivot, edge-centric, degeneracy order)",
        "value": m / (ms_per_step / 1e3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "chung_lu(n=%d, mean_deg=32, gamma=2.1, wmax=%.0f, seed=2)" % (g.n, wmax),
            "n": g.n, "m": m, "d_max": dag.d_max, "degeneracy": dag.degeneracy,
            "ks": ks, "order": "degeneracy", "scheme": "EC" if args.scheme == 2 else "VC",
            "validate": True,
        },
        "orient_ms": round(sum(orient_ms) / max(1, len(orient_ms)), 3),
        "per_k": per_k,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "literal_wmax20000": literal,
        "ablation_no_bitsets": ablation,
        "orientation_criteria": orders,
        "listing": listing,
        "small": small,
        "batched": batched,
        "dense_core": dense,
        "served": served,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
