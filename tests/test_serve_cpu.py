"""Serving loop logic on the CPU: admission by footprint, rejection of
oversized requests, the budget invariant under concurrency, and isolation of
a failing request.  The executor here is a stand-in (it computes the
oracle's global counts); the GPU test runs the real one."""

import threading
import time

import numpy as np

from paper_2010_14058_amd import serve as S
from tg_synth import graphs as G


def _req(rid, g, arrival=0.0):
    return S.Request(rid, g.row_ptr, g.col, g.types, g.L, arrival=arrival)


class FakeExecutor:
    def __init__(self, oracle_mod, delay=0.01, bad=()):
        self.oracle = oracle_mod
        self.delay = delay
        self.bad = set(bad)
        self.max_in_use = 0
        self.server = None
        self.lock = threading.Lock()
        self.calls = []

    def run(self, batch, w):
        with self.lock:
            self.calls.append([r.rid for r in batch])
            if self.server is not None:
                self.max_in_use = max(self.max_in_use, self.server.in_use)
        time.sleep(self.delay)
        if any(r.rid in self.bad for r in batch):
            err = RuntimeError("bad graph")
            err.code = 2
            raise err
        out = []
        for r in batch:
            g = G.Graph(r.row_ptr, r.col, r.types, r.L)
            out.append(self.oracle.global_counts(g, self.oracle.all_edge_rows(g, threads=1)))
        return out


def test_admission_budget_and_rejection(oracle_mod):
    graphs = [G.random_small_graph(12, 0.4, 3, s) for s in range(20)]
    ex = FakeExecutor(oracle_mod)
    srv = S.Server(hbm_budget=150, executor=ex, workers=2, footprint=lambda r: r.m + 10)
    ex.server = srv
    big = G.random_small_graph(30, 0.9, 2, 99)   # footprint (~400) > budget
    reqs = [_req(q, g) for q, g in enumerate(graphs)] + [_req(100, big)]
    for r in reqs:
        srv.submit(r)
    srv.close(timeout=60)
    rep = srv.report()
    assert rep["requests"] == 21 and rep["completed"] == 20 and rep["rejected"] == 1
    assert reqs[-1].status == S.TG_E_OOM
    assert ex.max_in_use <= 150 and srv.in_use == 0
    for r, g in zip(reqs, graphs):
        want = oracle_mod.global_counts(g, oracle_mod.all_edge_rows(g, threads=1))
        np.testing.assert_array_equal(r.result, want)
        assert r.t_admit >= 0 and r.t_done >= r.t_start >= r.t_admit
    # continuous batching: later requests were grouped while earlier ones ran
    assert max(len(c) for c in ex.calls) > 1


def test_failing_request_is_isolated(oracle_mod):
    graphs = [G.random_small_graph(10, 0.5, 2, 50 + s) for s in range(8)]
    ex = FakeExecutor(oracle_mod, delay=0.0, bad={3})
    srv = S.Server(hbm_budget=10**9, executor=ex, workers=1, footprint=lambda r: 1)
    reqs = [_req(q, g) for q, g in enumerate(graphs)]
    for r in reqs:
        srv.submit(r)
    srv.close(timeout=60)
    assert [r.status for r in reqs] == [0, 0, 0, 2, 0, 0, 0, 0]
    assert reqs[3].result is None and "bad graph" in reqs[3].error
    assert all(r.result is not None for q, r in enumerate(reqs) if q != 3)


def test_fifo_admission_no_overtaking(oracle_mod):
    graphs = [G.random_small_graph(10, 0.5, 2, 70 + s) for s in range(6)]
    ex = FakeExecutor(oracle_mod, delay=0.02)
    order = []
    srv = S.Server(hbm_budget=3, executor=ex, workers=2, footprint=lambda r: 1 if r.rid != 2 else 3,
                   uploader=lambda r: order.append(r.rid))
    for q, g in enumerate(graphs):
        srv.submit(_req(q, g))
    srv.close(timeout=60)
    assert order == list(range(6))
