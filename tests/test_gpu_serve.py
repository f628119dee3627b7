"""Serving on the GPU: requests arriving over time are batched continuously;
every result must be identical to the same graph counted alone."""

import numpy as np
import pytest

from tg_synth import graphs as G

pytestmark = pytest.mark.gpu


def test_results_identical_alone_and_in_mix(oracle_mod):
    from gpu_util import run_gpu
    from paper_2010_14058_amd import serve as S

    rng = np.random.default_rng(5)
    graphs = []
    for q in range(36):
        kind = q % 3
        if kind == 0:
            g = G.random_small_graph(int(rng.integers(5, 40)), float(rng.uniform(0.1, 0.7)),
                                     int(rng.integers(1, 9)), 300 + q)
        elif kind == 1:
            g = G.chung_lu_typed(int(rng.integers(200, 3000)), 10.0, 2.2, 150.0,
                                 int(rng.integers(2, 9)), seed=400 + q)
        else:
            g = G.er_graph(int(rng.integers(50, 500)), 6.0, 6, seed=500 + q)
        graphs.append(g)
    reqs = [S.Request(q, g.row_ptr, g.col, g.types, g.L, arrival=0.004 * q)
            for q, g in enumerate(graphs)]
    # one request with a self-loop: it alone must fail
    bad = graphs[7]
    rp = bad.row_ptr.copy()
    col = bad.col.copy()
    col[rp[0]] = 0 if rp[1] > rp[0] else col[rp[0]]
    reqs[7] = S.Request(7, rp, col, bad.types, bad.L, arrival=reqs[7].arrival)
    # requests of at least 2000 edges run as single-graph calls inside their batch
    ex = S.GpuExecutor(workers=2, single_edges=2000)
    srv = S.Server(hbm_budget=64 << 30, executor=ex, workers=2, max_batch_edges=20_000)
    print(f"[gpu] serving {len(reqs)} requests", flush=True)
    S.replay(srv, reqs)
    srv.close(timeout=120)
    rep = srv.report()
    print(rep, flush=True)
    assert rep["requests"] == len(reqs)
    assert srv.batches < len(reqs)           # requests were batched
    assert any(r.m >= 2000 for r in reqs) and any(r.m < 2000 for r in reqs)
    for q, (r, g) in enumerate(zip(reqs, graphs)):
        if q == 7:
            assert r.status == 2 and r.result is None
            continue
        assert r.status == 0, (q, r.error)
        _, alone = run_gpu(g)
        np.testing.assert_array_equal(r.result, alone, err_msg=f"request {q}")
        if g.m < 3000:
            want = oracle_mod.global_counts(g, oracle_mod.all_edge_rows(g, threads=8))
            np.testing.assert_array_equal(r.result, want)
