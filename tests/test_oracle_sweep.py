"""The oracle against the template brute force on 10^4 random typed graphs
(n 4..10, L 1..4, every density), rows in both orientations and global
instance counts, and its position-aware rows on 2,000 of them; the graphs
are spread over worker processes."""

import concurrent.futures as cf
import os

import numpy as np

import brute_force as BF
from tg_synth import graphs as G

COUNT = 10_000
PA_EVERY = 5


def _check(start: int, stop: int) -> list:
    import oracle

    bad = []
    for s in range(start, stop):
        rng = np.random.default_rng(70_000 + s)
        n = int(rng.integers(4, 11))
        L = int(rng.integers(1, 5))
        p = float(rng.uniform(0.05, 1.0))
        g = G.random_small_graph(n, p, L, 70_000 + s)
        uv = g.edges()
        if uv.shape[0] == 0:
            continue
        edges = [tuple(e) for e in uv.tolist()]
        want = BF.per_edge_rows(n, edges, g.types, L)
        for method in ("paper", "definition"):
            if not np.array_equal(oracle.edge_rows(g, uv, method=method, threads=1), want):
                bad.append((s, method))
            if not np.array_equal(oracle.edge_rows(g, uv[:, ::-1].copy(), method=method,
                                                   threads=1), want):
                bad.append((s, method + " reversed"))
        if not np.array_equal(oracle.global_counts(g, want),
                              BF.global_instances(n, edges, g.types, L)):
            bad.append((s, "global"))
        if s % PA_EVERY == 0:
            pa = BF.pa_per_edge_rows(n, edges, g.types, L)
            if not np.array_equal(oracle.pa_edge_rows(g, uv, threads=1), pa):
                bad.append((s, "position-aware"))
    return bad


def test_oracle_against_brute_force_sweep(oracle_mod):
    workers = max(1, min(8, os.cpu_count() or 1))
    step = 250
    bad = []
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        futs = [ex.submit(_check, a, min(a + step, COUNT)) for a in range(0, COUNT, step)]
        for f in futs:
            bad += f.result()
    assert not bad, bad[:10]
