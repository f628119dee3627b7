"""Benchmark: per-edge typed 3+4-node graphlet counts on one MI355X.

Workload: the Chung-Lu power-law graph (1M nodes, ~10M undirected edges,
degree exponent 2.1, largest degree ~5e4, L = 5 types with Zipf(1.2)
frequencies, same-type edge fraction 0.6), generated from seed 0.
One step = one full call of the library on that graph (input checks,
degree-rank relabelling, typed triangles, node aggregates, both 4-cycle
passes, cliques and derivation, the 12.8 GB per-edge table and the global
counts), with the graph already resident in HBM.

Prints one JSON line.  ``value`` is undirected edges per second over the
timed steps.  ``roofline`` covers the kernel with the largest average time
(HIP events on the library's stream), priced with the algorithmic bytes of
that kernel.  ``cpu_baseline`` is the CPU oracle (the paper's algorithm) on
a bounded random sample of the same graph's edges, timed on the host.

Scheduling knobs: a tuned profile ``paper_2010_14058_amd/tuned/<workload>.json``
(written by ``--autotune --tune-out PATH``) is applied when present and
reported under ``tuning``; ``--no-tuned`` keeps the library defaults.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure
CSRC = os.path.join(ROOT, "paper_2010_14058_amd", "csrc")
TUNED_DIR = os.path.join(ROOT, "paper_2010_14058_amd", "tuned")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    """Digest of every HIP source and header of the library."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def host_threads() -> int:
    """Worker threads for the CPU oracle: every CPU this process may run on,
    capped at 16 (the CPU share one GPU gets on the benchmark machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_info() -> dict:
    """CPU model, sockets, cores and threads of the host (lscpu), and the
    CPUs this process may use."""
    info = {}
    try:
        import subprocess

        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except Exception:  # lscpu missing: report what os says
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": info.get("Model name"), "sockets": info.get("Socket(s)"),
            "cores_per_socket": info.get("Core(s) per socket"),
            "threads_per_core": info.get("Thread(s) per core"), "cpus": info.get("CPU(s)"),
            "usable_cpus": usable, "oracle_threads": host_threads()}


def rank_order(d: np.ndarray) -> np.ndarray:
    """Node ids in the library's internal order: ascending (degree, id)."""
    ids = np.arange(d.size, dtype=np.int64)
    return np.lexsort((ids, d))


def ceil_log2p1(x: np.ndarray) -> np.ndarray:
    """Steps of a binary search over x entries: ceil(log2(x + 1))."""
    return np.ceil(np.log2(x.astype(np.float64) + 1.0))


def algorithmic_bytes(g, L, stats, members, members_heavy, edge_deg):
    """Bytes each kernel must move with no cache reuse, from this run's unit
    counts and the graph.

    Cycle passes: 8 B per wedge, 4 B to build (the target id read while
    counting) and 4 B to probe (the same target met again when emitting).
    Triangles and the triangle-set build: the shorter row of each edge is
    walked (4 B per entry and its 1-byte type) and each entry is probed in
    the other endpoint: one 8-byte bitmap word when that endpoint has a
    super-hub bitmap (or both are in the hub core), else a binary search of
    ceil(log2(d + 1)) 4-byte reads.  Clique walks are not priced (a lower
    bound).  Per-edge and per-node fixed reads and writes as listed."""
    n, m, nnz = g.n, g.m, g.nnz
    d = g.degrees().astype(np.int64)
    uv = g.edges()
    P = L * (L + 1) // 2
    W = 2 * L + 10 * P
    LP = (L + 3) & ~3
    LL = L * L
    narrow = int(d.max(initial=0)) < 65536
    aw = 4 if narrow else 8                 # word of A, D, NC and X_i, X_j, Y, K
    order = rank_order(d)
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    H = int(stats.get("hub_core", 0))
    S = int(stats.get("superhubs", 0))
    is_hub = rank >= n - H
    is_sh = rank >= n - S
    # hub-core neighbours per node
    src = np.repeat(np.arange(n), d)
    hubcnt = np.bincount(src, weights=is_hub[g.col].astype(np.float64), minlength=n)
    du, dv = d[uv[:, 0]], d[uv[:, 1]]
    s_is_u = du <= dv
    ds = np.where(s_is_u, du, dv).astype(np.float64)
    b = np.where(s_is_u, uv[:, 1], uv[:, 0])
    s = np.where(s_is_u, uv[:, 0], uv[:, 1])
    hs = hubcnt[s]
    bs = 4.0 * ceil_log2p1(d[b])
    probe = np.where(is_sh[b], 8.0 * ds,
                     np.where(is_hub[b], 8.0 * hs + bs * (ds - hs), bs * ds))
    tri = float(np.sum(5.0 * ds + probe)) + m * (8 + 8 + 32 + 4 * L + 8 * LP)
    # triangle-set build: low prefixes (non-hub neighbours) walked and
    # probed, hub members from two bit rows or the shorter hub suffix
    low = d - hubcnt
    lu, lv = low[uv[:, 0]], low[uv[:, 1]]
    ls = np.minimum(lu, lv)
    lo_other = np.where(lu <= lv, uv[:, 1], uv[:, 0])
    lprobe = np.where(is_sh[lo_other], 8.0 * ls, 4.0 * ceil_log2p1(low[lo_other]) * ls)
    hw = 8 * (((H + 63) // 64 + 7) // 8) if H else 0
    both_hub = is_hub[uv[:, 0]] & is_hub[uv[:, 1]]
    hu, hv = hubcnt[uv[:, 0]], hubcnt[uv[:, 1]]
    hsmall = np.minimum(hu, hv)
    hpart = np.where(both_hub, 16.0 * hw, 5.0 * hsmall + 8.0 * hsmall)
    per_edge_build = 5.0 * ls + lprobe + hpart
    heavy = np.minimum(du, dv) > int(edge_deg)
    per_member = 12 * LP + 8                    # three gathered rows and two slots
    hv_share = float(np.sum(per_edge_build[heavy]))
    b_all = float(np.sum(per_edge_build))
    nh = int(heavy.sum())
    xyk = 4 * LL * aw
    wa, wah = stats["wedges_pass_a"], stats["heavy_wedges_pass_a"]
    wb, wbh = stats["wedges_pass_b"], stats["heavy_wedges_pass_b"]
    # heavy wedges of the blocked path (its own phase) and of the task kernel
    wak, wbk = stats.get("blocked_wedges_pass_a", 0), stats.get("blocked_wedges_pass_b", 0)
    out = {
        "prep": 8 * (n + 1) + 4 * nnz + n + 8 * (n + 1) + 8 * nnz + 8 * m + 4 * n * L,
        "tri": tri,
        "aggr": nnz * (4 + 1 + 8 * LP) + 2 * aw * n * LL,
        "cyc_work": 28 * nnz,
        "cycA_light": 8 * (wa - wah),
        "cycA_blk": 8 * wak,
        "cycA_heavy": 8 * (wah - wak),
        "cycB_light": 8 * (wb - wbh),
        "cycB_blk": 8 * wbk,
        "cycB_heavy": 8 * (wbh - wbk),
        "edges_light": (b_all - hv_share) + (members - members_heavy) * per_member
                       + (m - nh) * (xyk + 56),
        "edges_heavy": hv_share + members_heavy * per_member + nh * (xyk + 56),
        "derive": m * (5 * LL * aw + xyk + 4 * L + 8 * LP + 8 * W),
    }
    # map traffic beyond the 8 algorithmic bytes: per task-kernel wedge a
    # counter update and L counts read; per blocked wedge a 2-byte record
    # written and read, three more target reads and one map word
    scratch = {"cycA_heavy": (16 + 4 * L) * (wah - wak), "cycB_heavy": (16 + 4 * L) * (wbh - wbk),
               "cycA_blk": (2 + 2 + 12 + 4) * wak, "cycB_blk": (2 + 2 + 12 + 4) * wbk}
    return {k: float(v) for k, v in out.items()}, scratch


def setup_tuning(args, workload: str, run) -> dict:
    """Knobs for the timed run: tune now (--autotune), else the workload's
    tuned profile when there is one, else the library defaults."""
    import paper_2010_14058_amd as P
    from paper_2010_14058_amd import autotune as AT

    path = os.path.join(TUNED_DIR, workload + ".json")
    if args.autotune:
        space = AT.BATCH_SPACE if args.mode == "batch" else AT.SINGLE_SPACE
        log(f"[bench] autotuning {len(space)} knobs on {workload}")
        res = AT.tune(run, space, min_gain=args.tune_min_gain, log=log)
        if args.tune_out:
            AT.save(res, args.tune_out, workload)
        return {"profile": "tuned in this run", "knobs": res.best,
                "start_ms": round(res.start_ms, 3), "best_ms": round(res.best_ms, 3),
                "trials": len(res.trials)}
    if os.path.exists(path) and not args.no_tuned:
        prof = AT.load(path)
        AT.apply(prof)
        return {"profile": os.path.relpath(path, ROOT), "knobs": prof["knobs"]}
    return {"profile": None, "knobs": P.get_tuning()}


# Phases that are pipelines of kernels (their time is the sum of the launches).
MULTI_KERNEL_PHASES = {
    ph: [f"k_blk_{k}" for k in ("select", "setup", "items", "hist", "part", "count", "emit")]
    + ["k_scan_tiles", "k_scan_sums", "k_scan_apply"]
    for ph in ("cycA_blk", "cycB_blk")}


def load_traffic(kernel: str):
    """Measured HBM bytes per launch of `kernel`, if recorded for this source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != kernel_source_sha():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(g, threads, target_s=15.0, seed=123):
    import oracle

    uv = g.edges()
    rng = np.random.default_rng(seed)
    k = 256
    pick = rng.choice(uv.shape[0], size=k, replace=False)
    t0 = time.perf_counter()
    oracle.edge_rows(g, uv[pick], method="paper", threads=threads)
    dt = time.perf_counter() - t0
    k2 = int(min(uv.shape[0], max(k, k * target_s / max(dt, 1e-3))))
    k2 = min(k2, 400_000)
    pick = np.sort(rng.choice(uv.shape[0], size=k2, replace=False))
    t0 = time.perf_counter()
    rows = oracle.edge_rows(g, uv[pick], method="paper", threads=threads)
    dt = time.perf_counter() - t0
    return pick, rows, {
        "value": k2 / dt,
        "unit": "edges/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{k2} edges drawn uniformly at random (seed {seed}) from the workload graph; "
                   f"the paper's per-edge algorithm (Alg. 1-3 with Lemmas 1-4) on {threads} "
                   f"threads; {dt:.1f} s"),
    }


def run_batch_workload(args, graphs: int, single_sample: int, oracle_graphs: int, steps: int,
                       tune: bool = True):
    """The batched configuration: 1e5 small typed Chung-Lu graphs counted by
    one call (eagerly, and replayed from a HIP graph recorded from the call
    without host synchronisation), against the same graphs counted one call
    per graph."""
    import torch

    import oracle
    import paper_2010_14058_amd as P
    from tg_synth import graphs as G

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    b = G.batch_graphs(graphs, seed=0)
    u = b.union
    gen_s = time.perf_counter() - t0
    log(f"[bench] batch of {b.G} graphs: n={u.n} m={u.m} max_degree={int(u.degrees().max())} "
        f"L_max={u.L} ({gen_s:.1f}s)")
    plan = P.BatchPlan(torch.from_numpy(u.row_ptr).to(dev), torch.from_numpy(u.col).to(dev),
                       torch.from_numpy(u.types).to(dev), b.node_ptr, b.L)
    ws = P.Workspace(dev)
    glob = torch.empty(int(plan.goff_host[-1]), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def run_once():
        from paper_2010_14058_amd import autotune as AT

        P.count_batch(plan, out_globals=glob, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        return AT.digest_of(glob)

    defaults = P.get_tuning()
    if tune:
        tuning = setup_tuning(args, G.CONFIG_NAMES[4], run_once)
    else:
        from paper_2010_14058_amd import autotune as AT

        path = os.path.join(TUNED_DIR, G.CONFIG_NAMES[4] + ".json")
        tuning = {"profile": None, "knobs": P.get_tuning()}
        if os.path.exists(path) and not args.no_tuned:
            prof = AT.load(path)
            AT.apply(prof)
            tuning = {"profile": os.path.relpath(path, ROOT), "knobs": prof["knobs"]}
    # eager calls (the call checks its inputs and reads the status back)
    P.set_timing(True)
    P.count_batch(plan, out_globals=glob, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    phase_sum = {}
    t_start = time.perf_counter()
    for _ in range(steps):
        P.count_batch(plan, out_globals=glob, workspace=ws, stream=stream)
        for name, ms in P.phase_times():
            phase_sum[name] = phase_sum.get(name, 0.0) + ms
    torch.cuda.synchronize()
    eager_s = time.perf_counter() - t_start
    P.set_timing(False)
    eager = glob.cpu().numpy().view(np.uint64).copy()
    stats = P.last_stats()
    # the same call recorded into a HIP graph and replayed
    out = torch.full_like(glob, -1)
    status = torch.full((1,), -1, dtype=torch.int32, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.count_batch_async(plan, out, status, ws, side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.count_batch_async(plan, out, status, ws, torch.cuda.current_stream())
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_r = time.perf_counter()
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    replay_s = time.perf_counter() - t_r
    replay_ev_ms = e0.elapsed_time(e1) / steps
    replay_ok = int(status.item()) == 0 and np.array_equal(out.cpu().numpy().view(np.uint64), eager)
    del graph
    log(f"[bench] batch: eager {eager_s * 1e3 / steps:.1f} ms per call, replay "
        f"{replay_s * 1e3 / steps:.1f} ms per launch, identical={replay_ok}")
    # the same graphs, one library call each (a prefix of the batch)
    S = min(single_sample, b.G)
    singles = []
    for g in range(S):
        gg = b.graph(g)
        singles.append((torch.from_numpy(gg.row_ptr).to(dev), torch.from_numpy(gg.col).to(dev),
                        torch.from_numpy(gg.types).to(dev), gg.L))
    sws = P.Workspace(dev)
    outs = [torch.empty(P.global_width(L), dtype=torch.int64, device=dev) for *_, L in singles]
    for q in range(min(50, S)):
        rp, col, ty, L = singles[q]
        P.count_typed_graphlets(rp, col, ty, L, per_edge=False, out_global=outs[q], workspace=sws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for q in range(S):
        rp, col, ty, L = singles[q]
        P.count_typed_graphlets(rp, col, ty, L, per_edge=False, out_global=outs[q], workspace=sws)
    torch.cuda.synchronize()
    single_s = time.perf_counter() - t1
    same = all(np.array_equal(outs[q].cpu().numpy().view(np.uint64),
                              eager[plan.goff_host[q]:plan.goff_host[q + 1]]) for q in range(S))
    single_gps = S / single_s
    res = {
        "workload": G.CONFIG_NAMES[4], "graphs": b.G, "n": u.n, "m": u.m, "L_max": int(u.L),
        "max_degree": int(u.degrees().max()), "generation_s": round(gen_s, 2),
        "replay_graphs_per_s": b.G * steps / replay_s,
        "replay_ms_per_launch_events": replay_ev_ms,
        "replay_identical_to_eager": bool(replay_ok),
        "eager_graphs_per_s": b.G * steps / eager_s,
        "eager_ms_per_call": eager_s * 1e3 / steps,
        "edges_per_s_replay": u.m * steps / replay_s,
        "single_call_path": {"graphs_per_s": single_gps, "graphs_timed": S,
                             "identical_counts": bool(same)},
        "speedup_replay_vs_single_call": (b.G * steps / replay_s) / single_gps,
        "tuning": tuning,
        "phases_ms": {k: round(v / steps, 3) for k, v in phase_sum.items()},
        "work": {k: int(v) for k, v in stats.items()},
    }
    if oracle_graphs > 0:
        k = min(b.G, oracle_graphs)
        t2 = time.perf_counter()
        ok = True
        for g in range(k):
            gg = b.graph(g)
            rows = oracle.edge_rows(gg, gg.edges(), method="paper", threads=1)
            want = oracle.global_counts(gg, rows)
            ok &= bool(np.array_equal(want, eager[plan.goff_host[g]:plan.goff_host[g + 1]]))
        dt = time.perf_counter() - t2
        res["cpu_baseline"] = {"value": k / dt, "unit": "graphs/s", "cores": 1, "kind": "oracle",
                               "sample": f"the first {k} graphs of the batch, paper algorithm, "
                                         f"one thread, {dt:.1f} s"}
        res["parity_sample"] = f"{k} graphs' global vectors identical to the oracle: {ok}"
        log(f"[bench] {res['parity_sample']}")
    P.set_tuning(**defaults)
    del plan, ws, glob, out, sws, singles, outs
    torch.cuda.empty_cache()
    return res


def bench_batch(args):
    res = run_batch_workload(args, args.graphs, args.single_sample, 4000, args.steps)
    result = {
        "metric": "batched graphs/sec (typed 3+4-node counts)",
        "value": res["replay_graphs_per_s"],
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": 1e3 * res["graphs"] / res["replay_graphs_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": res["workload"], "graphs": res["graphs"], "n": res["n"],
                   "m": res["m"], "L_max": res["L_max"], "max_degree": res["max_degree"]},
    }
    result.update({k: v for k, v in res.items() if k not in result["config"]})
    print(json.dumps(result), flush=True)


def run_serve_workload(args, requests: int, pool: int, rate: float, workers: int,
                       budget_gb: float, single_edges: int, max_batch_edges: int):
    """The serving configuration: a Poisson stream of `requests` requests at
    `rate` per second, each one typed Chung-Lu graph (edges log-uniform in
    [1e2, 1e6], n = m/5, exponent 2.2, L = 6 with Zipf(1.2) types) drawn from
    a pool of `pool` generated graphs, served by the native server (admission
    by HBM footprint, continuous batching on `workers` streams); against the
    pool's graphs counted one call each."""
    import torch

    import paper_2010_14058_amd as P
    from paper_2010_14058_amd import serve as S
    from tg_synth import graphs as G

    t0 = time.perf_counter()
    specs = G.serving_requests(pool, rate=rate, seed=0)
    graphs = [G.serving_graph(sp) for sp in specs]
    rng = np.random.default_rng(np.random.SeedSequence(1).spawn(1)[0])
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=requests))
    pick = rng.integers(0, pool, size=requests)
    reqs = [S.Request(q, graphs[k].row_ptr, graphs[k].col, graphs[k].types, graphs[k].L,
                      arrival=float(arrivals[q])) for q, k in enumerate(pick)]
    offered_edges = sum(r.m for r in reqs)
    span = float(arrivals[-1]) if requests else 1.0
    gen_s = time.perf_counter() - t0
    log(f"[bench] serving: {requests} requests from a pool of {pool} graphs, {offered_edges} "
        f"edges, arrivals over {span:.2f}s ({gen_s:.1f}s to generate)")
    defaults = P.get_tuning()
    path = os.path.join(TUNED_DIR, G.CONFIG_NAMES[4] + ".json")
    if os.path.exists(path) and not args.no_tuned:
        from paper_2010_14058_amd import autotune as AT

        AT.apply(AT.load(path))          # the batch profile for the workers
    srv = S.Server(hbm_budget=int(budget_gb * (1 << 30)), workers=workers,
                   single_edges=single_edges, max_batch_edges=max_batch_edges)
    S.replay(srv, reqs)
    srv.close()
    rep = srv.report()
    del srv
    import gc

    gc.collect()                 # the arena must be gone before the plain path is timed
    torch.cuda.empty_cache()
    P.set_tuning(**defaults)
    log(f"[bench] serving report: {rep}")
    # the plain path: the pool's graphs, one library call each
    dev = torch.device("cuda:0")
    ws = P.Workspace(dev)
    dev_graphs = [(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(g.types).to(dev), g.L) for g in graphs]
    P.count_typed_graphlets(*dev_graphs[0][:3], dev_graphs[0][3], per_edge=False, workspace=ws)
    torch.cuda.synchronize()
    outs = []
    t1 = time.perf_counter()
    for rp, col, ty, L in dev_graphs:
        _, g1 = P.count_typed_graphlets(rp, col, ty, L, per_edge=False, workspace=ws)
        outs.append(g1)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t1
    pool_edges = sum(g.m for g in graphs)
    by_pool = {}
    for r, k in zip(reqs, pick):
        if r.status == 0:
            by_pool.setdefault(int(k), r.result)
    same = all(np.array_equal(outs[k].cpu().numpy().view(np.uint64), res)
               for k, res in by_pool.items())
    all_same = all(np.array_equal(r.result, by_pool[int(k)]) for r, k in zip(reqs, pick)
                   if r.status == 0)
    plain = {"edges_per_s": pool_edges / plain_s, "graphs_per_s": pool / plain_s,
             "seconds": plain_s, "graphs": pool, "identical_counts": bool(same and all_same)}
    log(f"[bench] plain one-call-per-graph path: {plain}")
    del ws, dev_graphs, outs
    torch.cuda.empty_cache()
    return {
        "workload": G.CONFIG_NAMES[5], "requests": requests, "graph_pool": pool,
        "rate_per_s": rate, "workers": workers, "hbm_budget_GB": budget_gb,
        "max_batch_edges": max_batch_edges, "single_edges": single_edges,
        "served_edges_per_s": rep["served_edges_per_s"],
        "served_graphs_per_s": rep["served_graphs_per_s"],
        "offered_edges_per_s": offered_edges / max(span, 1e-9),
        "offered_requests_per_s": requests / max(span, 1e-9),
        "p50_latency_ms": rep["p50_latency_ms"], "p99_latency_ms": rep["p99_latency_ms"],
        "plain_path": plain,
        "speedup_vs_plain": {"edges": rep["served_edges_per_s"] / plain["edges_per_s"],
                             "graphs": rep["served_graphs_per_s"] / plain["graphs_per_s"]},
        "serving": rep, "generation_s": round(gen_s, 2),
    }


def bench_serve(args):
    res = run_serve_workload(args, args.requests, args.pool, args.rate, args.workers,
                             args.hbm_budget_gb, args.single_edges, args.max_batch_edges)
    result = {
        "metric": "served edges/sec (typed 3+4-node counts, Poisson arrivals)",
        "value": res["served_edges_per_s"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": res["requests"],
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": res["workload"], "requests": res["requests"],
                   "graph_pool": res["graph_pool"], "rate_per_s": res["rate_per_s"],
                   "workers": res["workers"], "hbm_budget_GB": res["hbm_budget_GB"]},
    }
    result.update({k: v for k, v in res.items() if k not in result["config"]})
    print(json.dumps(result), flush=True)


def stream_peak(dev, nbytes=1 << 31, reps=10) -> dict:
    """Measured streaming bandwidth of the device: a plain device-to-device
    copy of `nbytes`, timed with HIP events over `reps` copies (bytes read
    plus bytes written per copy)."""
    import torch

    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        b.copy_(a)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"GBps": 2 * nbytes / (ms * 1e-3) / 1e9, "copy_bytes": nbytes, "ms_per_copy": ms,
            "method": "device-to-device copy, read + write bytes over HIP-event time"}


def transfer_timings(g, rows, dev) -> dict:
    """Host-device transfer rates: the graph's input arrays to the device
    (pageable and pinned host memory) and a slice of the per-edge table back
    to pinned host memory (the full-table time is that rate applied to the
    table's size)."""
    import torch

    arrays = [g.row_ptr, g.col, g.types]
    nbytes = sum(a.nbytes for a in arrays)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [torch.from_numpy(a).to(dev) for a in arrays]
    torch.cuda.synchronize()
    pageable_s = time.perf_counter() - t0
    pinned = [torch.from_numpy(a).pin_memory() for a in arrays]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [p.to(dev, non_blocking=True) for p in pinned]
    torch.cuda.synchronize()
    pinned_s = time.perf_counter() - t0
    del outs, pinned
    res = {"h2d_input_bytes": nbytes, "h2d_pageable_ms": pageable_s * 1e3,
           "h2d_pageable_GBps": nbytes / pageable_s / 1e9, "h2d_pinned_ms": pinned_s * 1e3,
           "h2d_pinned_GBps": nbytes / pinned_s / 1e9}
    if rows is not None and rows.numel():
        k = max(1, min(rows.shape[0], (1 << 31) // (rows.shape[1] * 8)))
        host = torch.empty((k, rows.shape[1]), dtype=rows.dtype, pin_memory=True)
        host.copy_(rows[:k])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        host.copy_(rows[:k])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sl = k * rows.shape[1] * 8
        full = rows.shape[0] * rows.shape[1] * 8
        res.update({"d2h_slice_bytes": sl, "d2h_pinned_GBps": sl / dt / 1e9,
                    "d2h_full_table_ms_at_that_rate": full / (sl / dt) * 1e3})
        del host
    return res


def time_graph(P, torch, g, dev, steps, warmup, rows, glob, ws, stream, tag):
    """Warm-up calls, then `steps` timed calls of the library on g; returns
    wall-clock seconds, per-step event times and the per-phase averages."""
    L = g.L
    P.set_timing(True)
    for w in range(warmup):
        P.count_typed_graphlets(g._dev[0], g._dev[1], g._dev[2], L, out_rows=rows,
                                out_global=glob, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        log(f"[bench] {tag} warmup {w + 1}/{warmup} done")
    phase_sum = {}
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for q in range(steps):
        evs[q][0].record(stream)
        P.count_typed_graphlets(g._dev[0], g._dev[1], g._dev[2], L, out_rows=rows,
                                out_global=glob, workspace=ws, stream=stream)
        evs[q][1].record(stream)
        for name, ms in P.phase_times():
            phase_sum[name] = phase_sum.get(name, 0.0) + ms
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    step_ms = [a.elapsed_time(b) for a, b in evs]
    P.set_timing(False)
    return elapsed, step_ms, {k: v / max(steps, 1) for k, v in phase_sum.items()}


def roofline_of(P, torch, g, rows, stats, phase_avg, peak_stream):
    """Per-kernel algorithmic bytes and rates; the roofline entry of the
    kernel with the largest average time."""
    L = g.L
    uv = g.edges()
    d = g.degrees()
    edge_deg = P.get_tuning()["edge_deg"]
    hv = np.minimum(d[uv[:, 0]], d[uv[:, 1]]) > edge_deg
    hv_idx = torch.from_numpy(np.nonzero(hv)[0]).to(rows.device)
    members = float(stats["triangle_slots"])
    members_heavy = float(rows.index_select(0, hv_idx)[:, :L].sum().item()) if hv_idx.numel() else 0.0
    abytes, scratch = algorithmic_bytes(g, L, stats, members, members_heavy, edge_deg)
    kernels = [k for k in abytes if k != "prep" and k in phase_avg]
    # the blocked cycle phases are pipelines of several kernels (selection,
    # setup, item prefixes, histogram, partition, block counts, emit walk):
    # reported per phase, not as the dominant kernel
    single = [k for k in kernels if k not in MULTI_KERNEL_PHASES]
    per_kernel = {}
    over = []
    for k in kernels:
        gbps = abytes[k] / (phase_avg[k] * 1e-3) / 1e9 if phase_avg[k] > 0 else 0.0
        per_kernel[k] = {"ms": round(phase_avg[k], 3), "algorithmic_GB": round(abytes[k] / 1e9, 3),
                         "algorithmic_GBps": round(gbps, 1)}
        if gbps > HBM_PEAK_GBS:
            over.append(k)
    if over:
        log(f"[bench] WARNING: byte model above the HBM peak for {over}")
    dom = max(single, key=lambda k: phase_avg[k])
    dom_ms = phase_avg[dom]
    achieved = abytes[dom] / (dom_ms * 1e-3) / 1e9
    wak, wbk = stats.get("blocked_wedges_pass_a", 0), stats.get("blocked_wedges_pass_b", 0)
    units = {"cycA_heavy": ("wedge", stats["heavy_wedges_pass_a"] - wak),
             "cycB_heavy": ("wedge", stats["heavy_wedges_pass_b"] - wbk),
             "cycA_blk": ("wedge", wak), "cycB_blk": ("wedge", wbk)}.get(dom, ("edge", g.m))
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(dom),
            "avg_ms": dom_ms, "algorithmic_bytes_per_launch": abytes[dom],
            "work_unit": units[0], "units_per_launch": int(units[1]),
            "streaming_peak_GBps": peak_stream, "frac_of_streaming_peak":
                achieved / peak_stream if peak_stream else None,
            "streaming_peak_method": "device-to-device copy of 2 GiB, read + write bytes over "
                                     "HIP-event time"}
    if dom in scratch:
        roof["map_scratch_bytes_per_launch"] = scratch[dom]
    for k in MULTI_KERNEL_PHASES:
        if k in per_kernel:
            per_kernel[k]["kernels"] = MULTI_KERNEL_PHASES[k]
            per_kernel[k]["traffic"] = load_traffic(k)
            if k in scratch:
                per_kernel[k]["scratch_bytes"] = scratch[k]
    return roof, per_kernel, over, abytes


def parity_sample(g, rows, dev, k_uniform, per_hub, top, threads, seed):
    """Sampled rows of the GPU table against the oracle (uniform edges and
    edges at the top-degree nodes)."""
    import torch

    import oracle

    uv = g.edges()
    rng = np.random.default_rng(seed)
    pick = set(rng.choice(uv.shape[0], size=min(k_uniform, uv.shape[0]), replace=False).tolist())
    d = g.degrees()
    for h in np.argsort(-d, kind="stable")[:top]:
        inc = np.nonzero((uv[:, 0] == h) | (uv[:, 1] == h))[0]
        pick.update(rng.choice(inc, size=min(per_hub, inc.size), replace=False).tolist())
    pick = np.array(sorted(pick), dtype=np.int64)
    t0 = time.perf_counter()
    want = oracle.edge_rows(g, uv[pick], method="paper", threads=threads)
    dt = time.perf_counter() - t0
    got = rows.index_select(0, torch.from_numpy(pick).to(dev)).cpu().numpy().view(np.uint64)
    same = int(np.sum(np.all(got == want, axis=1)))
    return same, int(pick.size), dt


def bench_single(args):
    import torch

    import paper_2010_14058_amd as P
    from tg_synth import graphs as G

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    defaults = P.get_tuning()
    host = host_info()
    if args.calib_copy:
        # counter runs: the only device copy is the 1 GiB calibration copy
        peak = {"GBps": None, "method": "not measured in counter runs"}
    else:
        peak = stream_peak(dev)
        log(f"[bench] streaming copy: {peak['GBps']:.1f} GB/s")
    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("[bench] calibration copy of 1 GiB done")

    t0 = time.perf_counter()
    g = G.config_graph(2, seed=0, scale=args.scale)
    st = g.stats()
    gen_s = time.perf_counter() - t0
    log(f"[bench] graph {st['name']}: n={st['n']} m={st['m']} max_degree={st['max_degree']} "
        f"same_type={st['same_type_edge_fraction']:.4f} ({gen_s:.1f}s)")
    L = g.L
    g._dev = (torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
              torch.from_numpy(g.types).to(dev))
    W = P.row_width(L)
    rows = torch.empty((g.m, W), dtype=torch.int64, device=dev)
    glob = torch.empty(P.global_width(L), dtype=torch.int64, device=dev)
    ws = P.Workspace(dev)

    def run_once():
        from paper_2010_14058_amd import autotune as AT

        P.count_typed_graphlets(*g._dev, L, out_rows=rows, out_global=glob, workspace=ws,
                                stream=stream)
        torch.cuda.synchronize()
        return AT.digest_of(glob, rows)

    tuning = setup_tuning(args, st["name"], run_once)
    elapsed, step_ms, phase_avg = time_graph(P, torch, g, dev, args.steps, args.warmup, rows,
                                             glob, ws, stream, "power-law")
    log(f"[bench] {args.steps} timed steps in {elapsed:.3f}s")
    stats = P.last_stats()
    roof, per_kernel, over, abytes = roofline_of(P, torch, g, rows, stats, phase_avg,
                                                 peak["GBps"])
    ms_per_step = elapsed * 1e3 / args.steps
    result = {
        "metric": "edges/sec (typed 3+4-node counts)",
        "value": g.m * args.steps / elapsed,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": st["name"], "n": st["n"], "m": st["m"], "L": L,
                   "max_degree": st["max_degree"],
                   "same_type_edge_fraction": round(st["same_type_edge_fraction"], 4),
                   "per_edge_table_GB": round(g.m * W * 8 / 1e9, 2)},
        "roofline": roof,
        "ms_per_step_median_events": float(np.median(step_ms)),
        "step_ms_events": [round(x, 3) for x in step_ms],
        "kernels": per_kernel,
        "byte_model_above_peak": over,
        "pipeline_algorithmic_GBps": sum(abytes.values()) / (ms_per_step * 1e-3) / 1e9,
        "tuning": tuning,
        "phases_ms": {k: round(v, 3) for k, v in phase_avg.items()},
        "work": {k: int(v) for k, v in stats.items()},
        "host": host,
        "generation_s": round(gen_s, 2),
    }
    if not args.calib_copy:   # counter runs keep the calibration copy the only large copy
        result["transfers"] = transfer_timings(g, rows, dev)
        log(f"[bench] transfers: {result['transfers']}")

    # sparse per-edge form of the table (outside the timed steps)
    torch.cuda.synchronize()
    t_sp = time.perf_counter()
    off, keys, counts = P.sparse_rows(rows, L, workspace=ws)
    torch.cuda.synchronize()
    sp_ms = (time.perf_counter() - t_sp) * 1e3
    nnz_total = int(keys.numel())
    result["sparse_output"] = {
        "nonzeros": nnz_total, "mean_per_edge": nnz_total / max(g.m, 1),
        "bytes": nnz_total * 10 + (g.m + 1) * 8, "dense_bytes": g.m * W * 8,
        "ms": round(sp_ms, 3)}
    del off, keys, counts

    if not args.skip_cpu:
        threads = host_threads()
        log(f"[bench] CPU oracle baseline on {threads} threads ...")
        pick, orows, cb = cpu_baseline(g, threads)
        cb["sample"] += (f"; host {host['model']}, {host['sockets']} socket(s) x "
                         f"{host['cores_per_socket']} cores x {host['threads_per_core']} "
                         f"threads, {host['usable_cpus']} CPUs usable, oracle capped at 16 threads")
        result["cpu_baseline"] = cb
        sel = torch.from_numpy(pick).to(dev)
        grows = rows.index_select(0, sel).cpu().numpy().view(np.uint64)
        same = int(np.sum(np.all(grows == orows, axis=1)))
        result["parity_sample"] = f"{same}/{len(pick)} sampled rows identical to the oracle"
        log(f"[bench] {result['parity_sample']}")

    del rows, glob, g._dev
    ws.buf = None
    torch.cuda.empty_cache()
    if args.config3_steps > 0 and not args.no_extra:
        P.set_tuning(**defaults)
        result["config3"] = bench_config3(args, P, torch, G, dev, stream, peak["GBps"])
    if not args.no_extra:
        P.set_tuning(**defaults)
        result["position_aware"] = bench_position_aware(args, P, torch, G, dev, stream)
        result["directed"] = bench_directed(args, P, torch, G, dev, stream)
        result["embedding"] = bench_embedding(args, P, torch, G, dev, stream)
        result["batch"] = run_batch_workload(args, args.graphs, args.single_sample,
                                             0 if args.skip_cpu else 1000, 3, tune=False)
        result["serve"] = run_serve_workload(args, args.requests, args.pool, args.rate,
                                             args.workers, args.hbm_budget_gb, args.single_edges,
                                             args.max_batch_edges)
    print(json.dumps(result), flush=True)


def bench_config3(args, P, torch, G, dev, stream, peak_gbps):
    """The tripartite configuration at full size: edges/s, phases, roofline
    of its dominant kernel and a sampled parity check against the oracle."""
    t0 = time.perf_counter()
    g = G.config_graph(3, seed=0, scale=args.scale)
    st = g.stats()
    gen_s = time.perf_counter() - t0
    log(f"[bench] graph {st['name']}: n={st['n']} m={st['m']} max_degree={st['max_degree']} "
        f"({gen_s:.1f}s)")
    L = g.L
    g._dev = (torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
              torch.from_numpy(g.types).to(dev))
    rows = torch.empty((g.m, P.row_width(L)), dtype=torch.int64, device=dev)
    glob = torch.empty(P.global_width(L), dtype=torch.int64, device=dev)
    ws = P.Workspace(dev)
    elapsed, step_ms, phase_avg = time_graph(P, torch, g, dev, args.config3_steps, 1, rows, glob,
                                             ws, stream, "tripartite")
    stats = P.last_stats()
    roof, per_kernel, over, _ = roofline_of(P, torch, g, rows, stats, phase_avg, peak_gbps)
    out = {"workload": st["name"], "n": st["n"], "m": st["m"], "L": L,
           "max_degree": st["max_degree"], "steps": args.config3_steps, "warmup": 1,
           "value": g.m * args.config3_steps / elapsed, "unit": "edges/s",
           "ms_per_step": elapsed * 1e3 / args.config3_steps,
           "ms_per_step_median_events": float(np.median(step_ms)),
           "tuning": "library defaults", "roofline": roof, "kernels": per_kernel,
           "byte_model_above_peak": over,
           "phases_ms": {k: round(v, 3) for k, v in phase_avg.items()},
           "work": {k: int(v) for k, v in stats.items()}, "generation_s": round(gen_s, 2)}
    if not args.skip_cpu:
        same, k, dt = parity_sample(g, rows, dev, 64, 4, 8, host_threads(), 29)
        out["parity_sample"] = (f"{same}/{k} sampled rows (64 uniform edges, 4 at each of the "
                                f"8 highest-degree nodes) identical to the oracle; {dt:.1f} s")
        log(f"[bench] tripartite: {out['parity_sample']}")
    del rows, glob, g._dev
    ws.buf = None
    torch.cuda.empty_cache()
    return out


def bench_position_aware(args, P, torch, G, dev, stream, steps=3):
    """Position-aware typed counts (Sec. 5) of the headline power-law graph:
    per-edge rows (3L + 9L^2 + 6P columns) and global classes per step, and
    a sampled parity check of rows against the oracle."""
    import oracle   # parity sample only, outside the timed steps

    g = G.config_graph(2, seed=0, scale=args.scale)
    L = g.L
    rp, col, ty = (torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(g.types).to(dev))
    W = P.pa_row_width(L)
    rows = torch.empty((g.m, W), dtype=torch.int64, device=dev)
    glob = torch.empty(P.pa_global_width(L), dtype=torch.int64, device=dev)
    ws = P.Workspace(dev)
    P.count_position_aware(rp, col, ty, L, out_rows=rows, out_global=glob, workspace=ws,
                           stream=stream)                                  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        P.count_position_aware(rp, col, ty, L, out_rows=rows, out_global=glob, workspace=ws,
                               stream=stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"workload": g.name, "n": g.n, "m": g.m, "L": L, "row_width": W,
           "per_edge_table_GB": round(g.m * W * 8 / 1e9, 2), "steps": steps,
           "value": g.m * steps / el, "unit": "edges/s", "ms_per_step": el * 1e3 / steps,
           "global_classes_nonzero": int((glob != 0).sum())}
    uv = g.edges()
    rng = np.random.default_rng(5)
    deg = g.degrees()
    hub = np.flatnonzero(np.maximum(deg[uv[:, 0]], deg[uv[:, 1]]) > 5000)
    pick = np.unique(np.concatenate([rng.choice(g.m, 64, replace=False),
                                     rng.choice(hub, min(16, hub.size), replace=False)]))
    t1 = time.perf_counter()
    want = oracle.pa_edge_rows(g, uv[pick], threads=host_threads())
    got = rows.index_select(0, torch.from_numpy(pick).to(dev)).cpu().numpy().view(np.uint64)
    same = int(np.sum(np.all(got == want, axis=1)))
    out["parity_sample"] = (f"{same}/{len(pick)} sampled rows (64 uniform, 16 hub-incident) "
                            f"identical to the oracle; {time.perf_counter() - t1:.1f} s")
    log(f"[bench] position-aware: {out['value']:.3e} edges/s, {out['parity_sample']}")
    del rows, glob, rp, col, ty
    ws.buf = None
    torch.cuda.empty_cache()
    return out


def bench_directed(args, P, torch, G, dev, stream, steps=3):
    """Directed typed 3-node counts (Sec. 4.8) on the headline power-law
    graph with its edges oriented (20% reciprocal, else a fair coin): the
    whole call (checks, rows, global classes) per step, and a sampled parity
    check of rows against the oracle."""
    from oracle import directed as OD   # oracle: parity sample only, outside the timed steps

    g = G.config_graph(2, seed=0, scale=args.scale)
    dirs = G.orient(g, 0.2, 7)
    L = g.L
    rp, col, ty = (torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(g.types).to(dev))
    d = torch.from_numpy(dirs).to(dev)
    ws = P.Workspace(dev)
    P.count_directed(rp, col, d, ty, L, workspace=ws, stream=stream)      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rows, glob = P.count_directed(rp, col, d, ty, L, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # algorithmic bytes of the row pass: the row write, the shorter adjacency
    # list (ids and direction bytes) and both endpoints' direction-split degrees
    deg = g.degrees()
    uv = g.edges()
    shorter = np.minimum(deg[uv[:, 0]], deg[uv[:, 1]]).astype(np.int64)
    abytes = g.m * (15 * L * 8 + 2 * 3 * L * 4 + 16) + int(shorter.sum()) * 5
    # one more call with per-kernel HIP events (outside the timed steps)
    P.set_timing(True)
    rows, glob = P.count_directed(rp, col, d, ty, L, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    ks = P.kernel_sums()
    P.set_timing(False)
    rows_ms = ks.get("dir_rows", {}).get("ms", 0.0)
    roof = None
    if rows_ms > 0:
        ach = abytes / (rows_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "k_dir_rows", "achieved": ach, "peak": 8000.0,
                "unit": "GB/s", "frac": ach / 8000.0, "traffic": None, "avg_ms": rows_ms,
                "algorithmic_bytes_per_launch": abytes, "work_unit": "edge",
                "units_per_launch": g.m}
    out = {"workload": g.name + " oriented (20% reciprocal)", "n": g.n, "m": g.m, "L": L,
           "steps": steps, "value": g.m * steps / el, "unit": "edges/s",
           "ms_per_step": el * 1e3 / steps,
           "algorithmic_bytes_per_step": abytes,
           "pipeline_algorithmic_GBps": abytes / (el / steps) / 1e9,
           "roofline": roof,
           "kernels_ms": {k: round(v["ms"], 3) for k, v in ks.items()},
           "global_classes_nonzero": int((glob != 0).sum())}
    rng = np.random.default_rng(3)
    pick = rng.choice(g.m, 500, replace=False)
    grows = rows.index_select(0, torch.from_numpy(pick).to(dev)).cpu().numpy().view(np.uint64)
    same = sum(int(np.array_equal(grows[q], OD.edge_row(g, dirs, int(uv[e, 0]), int(uv[e, 1]))))
               for q, e in enumerate(pick.tolist()))
    out["parity_sample"] = f"{same}/500 sampled rows identical to the oracle"
    log(f"[bench] directed: {out['value']:.3e} edges/s, {out['parity_sample']}")
    del rows, glob, rp, col, ty, d
    ws.buf = None
    torch.cuda.empty_cache()
    return out


def bench_embedding(args, P, torch, G, dev, stream):
    """Alg. 5 embeddings of the headline power-law graph for a few typed
    graphlets: weights from the per-edge rows, then the per-component
    solve; seconds, iterations and component sizes per case."""
    g = G.config_graph(2, seed=0, scale=args.scale)
    L = g.L
    rp, col, ty = (torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(g.types).to(dev))
    ws = P.Workspace(dev)
    rows, _ = P.count_typed_graphlets(rp, col, ty, L, workspace=ws, stream=stream)
    uv = P.edge_list(rp, col, workspace=ws, stream=stream)
    cases = [(2, (0, 0, 0), 16), (1, (0, 0, 1), 16), (5, (0, 0, 1, 1), 16), (1, (0, 0, 1), 128),
             (0, (0, 1), 128)]
    weights = {}
    torch.cuda.synchronize()
    for h, ms, _ in cases:
        if (h, ms) not in weights:
            t0 = time.perf_counter()
            weights[(h, ms)] = P.graphlet_weights(rows, uv, ty, L, h, ms, stream=stream)
            torch.cuda.synchronize()
            log(f"[bench] weights h{h} {ms}: {1e3 * (time.perf_counter() - t0):.2f} ms")
    del rows, uv
    ws.buf = None
    torch.cuda.empty_cache()
    out = []
    P.set_timing(True)          # per-kernel-class HIP events (a few microseconds per launch)
    for h, ms, dim in cases:
        w = weights[(h, ms)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Z, ev, comp, its = P.graphlet_embedding(rp, col, w, dim, workspace=ws, stream=stream,
                                                check=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ks = P.kernel_sums()
        c = comp.cpu().numpy()
        sizes = np.bincount(c[c >= 0]) if (c >= 0).any() else np.zeros(1, dtype=np.int64)
        sizes = sizes[sizes > 0]
        rec = {"graphlet": f"h{h}", "types": list(ms), "dim": dim, "seconds": round(el, 3),
               "iterations": its, "converged": bool(its < 500),
               "weighted_edges": int((w != 0).sum()), "components": int(sizes.size),
               "largest_component": int(sizes.max()) if sizes.size else 0,
               "components_over_64": int((sizes > 64).sum()),
               "kernels_ms": {k: round(v["ms"], 2) for k, v in ks.items()}}
        sp = ks.get("spmm")
        if sp and sp["ms"] > 0:
            rec["spmm_GBps"] = round(sp["units"] / (sp["ms"] * 1e-3) / 1e9, 1)
        mf = [ks[k] for k in ("gram", "apply") if k in ks and ks[k]["ms"] > 0]
        if mf:
            rec["mfma_TFLOPs"] = round(sum(v["units"] for v in mf) /
                                       (sum(v["ms"] for v in mf) * 1e-3) / 1e12, 2)
        if dim == 128 and h == 1 and sp and sp["ms"] > 0:
            ach = sp["units"] / (sp["ms"] * 1e-3) / 1e9
            rec["roofline"] = {"bound": "hbm", "kernel": "k_spmm_rows/items/finish",
                               "achieved": ach, "peak": 8000.0, "unit": "GB/s",
                               "frac": ach / 8000.0, "traffic": None,
                               "avg_ms": sp["ms"] / max(sp["calls"], 1),
                               "algorithmic_bytes_per_launch": sp["units"] / max(sp["calls"], 1),
                               "work_unit": "nonzero of S (12 + 8p bytes) and block row"}
            if mf:
                fl = sum(v["units"] for v in mf)
                t = sum(v["ms"] for v in mf) * 1e-3
                rec["roofline_mfma"] = {"bound": "mfma", "kernel": "k_emb_gram_part + k_emb_apply",
                                        "achieved": fl / t / 1e12, "peak": 78.6,
                                        "unit": "TFLOP/s", "frac": fl / t / 1e12 / 78.6,
                                        "traffic": None, "dtype": "f64"}
        out.append(rec)
        log(f"[bench] embedding {rec}")
        del Z, ev, comp
    P.set_timing(False)
    ws.buf = None
    torch.cuda.empty_cache()
    return {"workload": g.name, "n": g.n, "m": g.m, "L": L, "tolerance": 1e-10,
            "method": "per component: dense Jacobi up to 64 nodes, else Chebyshev-filtered "
                      "subspace iteration (float64)", "cases": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=["single", "batch", "serve", "directed", "embedding",
                                       "position_aware"],
                    default="single",
                    help="single: the 10M-edge power-law graph (headline); batch: 1e5 small "
                         "graphs in one call; serve: Poisson request stream")
    ap.add_argument("--requests", type=int, default=20000, help="serve mode: number of requests")
    ap.add_argument("--pool", type=int, default=400,
                    help="serve mode: distinct graphs the requests are drawn from")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve mode: arrivals per second")
    ap.add_argument("--workers", type=int, default=4, help="serve mode: concurrent batches")
    ap.add_argument("--single-edges", type=int, default=1 << 17,
                    help="serve mode: requests with at least this many edges run as single calls")
    ap.add_argument("--hbm-budget-gb", type=float, default=160.0, help="serve mode: admission budget")
    ap.add_argument("--max-batch-edges", type=int, default=8_000_000,
                    help="serve mode: edges per batch at most")
    ap.add_argument("--graphs", type=int, default=100_000, help="batch mode: number of graphs")
    ap.add_argument("--single-sample", type=int, default=2000,
                    help="batch mode: graphs timed with one call each")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (testing only)")
    ap.add_argument("--skip-cpu", action="store_true", help="no CPU baseline (profiling runs)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the scheduling knobs on this workload before timing")
    ap.add_argument("--tune-out", default=None, help="with --autotune: write the profile here")
    ap.add_argument("--tune-min-gain", type=float, default=0.02,
                    help="with --autotune: least relative gain that changes a knob")
    ap.add_argument("--no-tuned", action="store_true",
                    help="ignore the tuned profile, time the library defaults")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--no-extra", action="store_true",
                    help="single mode: only the headline graph (no tripartite, batch or serving "
                         "summaries)")
    ap.add_argument("--config3-steps", type=int, default=3,
                    help="single mode: timed steps of the full-size tripartite graph after the "
                         "headline (0 skips it)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(this build has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    if args.mode == "batch":
        bench_batch(args)
        return
    if args.mode == "serve":
        bench_serve(args)
        return
    if args.mode in ("directed", "embedding", "position_aware"):
        # one extra leg alone (profiling runs): its summary as the JSON line
        import torch

        import paper_2010_14058_amd as P
        from tg_synth import graphs as G

        dev = torch.device("cuda:0")
        stream = torch.cuda.current_stream(dev)
        leg = {"directed": bench_directed, "embedding": bench_embedding,
               "position_aware": bench_position_aware}[args.mode]
        print(json.dumps({args.mode: leg(args, P, torch, G, dev, stream)}), flush=True)
        return

    bench_single(args)


if __name__ == "__main__":
    main()
