"""Serving on the GPU through the native server: requests arriving over time
are batched continuously; every result must be identical to the same graph
counted alone (and to the oracle for the small ones), a failing request
fails alone, device-resident inputs work, admission waits for memory, and
the server's errors are reported through its C calls."""

import ctypes

import numpy as np
import pytest

from tg_synth import graphs as G

pytestmark = pytest.mark.gpu


def _mixed_requests(S, count, seed):
    rng = np.random.default_rng(seed)
    graphs = []
    for q in range(count):
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
    # bursts of 6 requests 20 ms apart: a burst arrives within microseconds,
    # faster than any request is served, so requests always meet in a batch
    reqs = [S.Request(q, g.row_ptr, g.col, g.types, g.L, arrival=0.02 * (q // 6))
            for q, g in enumerate(graphs)]
    return graphs, reqs


def test_results_identical_alone_and_in_mix(oracle_mod):
    from gpu_util import run_gpu
    from paper_2010_14058_amd import serve as S

    graphs, reqs = _mixed_requests(S, 36, 5)
    # one request with a self-loop: it alone must fail
    bad = graphs[7]
    rp = bad.row_ptr.copy()
    col = bad.col.copy()
    col[rp[0]] = 0 if rp[1] > rp[0] else col[rp[0]]
    reqs[7] = S.Request(7, rp, col, bad.types, bad.L, arrival=reqs[7].arrival)
    # requests of at least 2000 edges run as single-graph calls
    srv = S.Server(hbm_budget=8 << 30, workers=2, single_edges=2000, max_batch_edges=20_000)
    print(f"[gpu] serving {len(reqs)} requests", flush=True)
    S.replay(srv, reqs)
    srv.close(timeout=120)
    rep = srv.report()
    print(rep, flush=True)
    assert rep["requests"] == len(reqs)
    assert rep["batches"] < len(reqs)           # requests were batched
    assert rep["single_calls"] >= 1
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


def test_admission_waits_for_memory(oracle_mod):
    """A pool of 1 MiB holds only a few requests at a time: the rest wait,
    and every request still finishes with the right counts."""
    from paper_2010_14058_amd import serve as S

    graphs, reqs = _mixed_requests(S, 30, 11)
    for r in reqs:
        r.arrival = 0.0
    wb = 512 << 20
    srv = S.Server(hbm_budget=wb + (1 << 20), workers=1, worker_bytes=wb, single_edges=1 << 30)
    S.replay(srv, reqs)
    srv.close(timeout=120)
    st = srv.stats
    assert st["finished"] == len(reqs) and st["peak_pool_bytes"] <= st["pool_bytes"]
    for r, g in zip(reqs, graphs):
        assert r.status == 0, r.error
        want = oracle_mod.global_counts(g, oracle_mod.all_edge_rows(g, threads=8))
        np.testing.assert_array_equal(r.result, want)


def test_device_inputs_and_errors():
    import torch

    import paper_2010_14058_amd as P
    from gpu_util import to_device
    from paper_2010_14058_amd import _lib

    lib = _lib.load()
    arena = torch.empty((1 << 30) + (4 << 20), dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    assert lib.tg_server_create(arena.data_ptr() + 1, arena.numel() - 256, 1, 1 << 30, 100, 10**6,
                                ctypes.byref(h)) == 1        # unaligned arena
    assert lib.tg_server_create(arena.data_ptr(), arena.numel(), 1, arena.numel(), 100, 10**6,
                                ctypes.byref(h)) == 10       # no pool left
    assert lib.tg_server_create(arena.data_ptr(), arena.numel(), 1, 1 << 30, 100, 10**6,
                                ctypes.byref(h)) == 0
    g = G.chung_lu_typed(2000, 8.0, 2.2, 100.0, 4, seed=3)
    rp, col, ty = to_device(g)
    desc = _lib.GraphDesc(rp.data_ptr(), col.data_ptr(), ty.data_ptr(), g.n, g.nnz, g.L, 1)
    t = ctypes.c_int64()
    assert lib.tg_server_submit(h, ctypes.byref(desc), ctypes.byref(t)) == 0
    assert lib.tg_server_wait(h, t.value, 60.0) == 0
    info = _lib.RequestInfo()
    assert lib.tg_server_poll(h, t.value, ctypes.byref(info)) == 0
    assert info.state == 3 and info.status == 0 and info.global_counts
    off = info.global_counts - arena.data_ptr()
    got = arena[off:off + 8 * P.global_width(g.L)].cpu().numpy().view(np.uint64)
    _, want = P.count_typed_graphlets(rp, col, ty, g.L, per_edge=False)
    np.testing.assert_array_equal(got, want.cpu().numpy().view(np.uint64))
    assert info.t_submit <= info.t_admit <= info.t_start <= info.t_done
    assert lib.tg_server_release(h, t.value) == 0
    assert lib.tg_server_release(h, t.value) == 1            # already released
    assert lib.tg_server_poll(h, 999, ctypes.byref(info)) == 1
    # a request whose block exceeds the whole pool
    n_big = 1_000_000                                        # an 8 MB row array alone
    big_rp = np.zeros(n_big + 1, dtype=np.int64)
    big_ty = np.zeros(n_big, dtype=np.uint8)
    bdesc = _lib.GraphDesc(big_rp.ctypes.data, 0, big_ty.ctypes.data, n_big, 0, 3, 0)
    assert lib.tg_server_submit(h, ctypes.byref(bdesc), ctypes.byref(t)) == 10
    assert lib.tg_server_destroy(h) == 0
