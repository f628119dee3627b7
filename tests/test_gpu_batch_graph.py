"""The batch entry point without host synchronisation, eagerly and recorded
into a HIP graph: every replay (with eager work and synchronisations
between replays) must give, for every graph, the oracle's counts and a
TG_OK status; input errors are reported through the device status word
without any kernel leaving its bounds."""

import numpy as np
import pytest

from tg_synth import graphs as G

pytestmark = pytest.mark.gpu


def _plan(b):
    import torch

    import paper_2010_14058_amd as P

    dev = torch.device("cuda:0")
    u = b.union
    return P.BatchPlan(torch.from_numpy(u.row_ptr).to(dev), torch.from_numpy(u.col).to(dev),
                       torch.from_numpy(u.types).to(dev), b.node_ptr, b.L)


def _expected(oracle_mod, b):
    out = []
    for g in range(b.G):
        gg = b.graph(g)
        out.append(oracle_mod.global_counts(gg, oracle_mod.all_edge_rows(gg, threads=4)))
    return np.concatenate(out)


def _buffers(plan):
    import torch

    import paper_2010_14058_amd as P

    dev = plan.row_ptr.device
    ws = P.Workspace(dev)
    ws.get(P.batch_workspace_bytes(plan.n, plan.nnz, plan.G, plan.L_max))
    out = torch.full((int(plan.goff_host[-1]),), -1, dtype=torch.int64, device=dev)
    status = torch.full((1,), -7, dtype=torch.int32, device=dev)
    return ws, out, status


def test_async_batch_matches_oracle(oracle_mod):
    import torch

    import paper_2010_14058_amd as P

    b = G.batch_graphs(400, seed=3)
    print(f"[gpu] async batch of {b.G} graphs, n={b.union.n} m={b.union.m}", flush=True)
    plan = _plan(b)
    ws, out, status = _buffers(plan)
    P.count_batch_async(plan, out, status, ws, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint64), _expected(oracle_mod, b))


def test_batch_graph_replays(oracle_mod):
    import torch

    import paper_2010_14058_amd as P

    b = G.batch_graphs(400, seed=3)
    want = _expected(oracle_mod, b)
    plan = _plan(b)
    ws, out, status = _buffers(plan)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):          # warm-up call outside the capture
        P.count_batch_async(plan, out, status, ws, side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    graph = torch.cuda.CUDAGraph()
    print("[gpu] capturing the batch call", flush=True)
    with torch.cuda.graph(graph):
        P.count_batch_async(plan, out, status, ws, torch.cuda.current_stream())
    torch.cuda.synchronize()
    other = G.batch_graphs(50, seed=8)
    oplan = _plan(other)
    for rep in range(4):
        # eager work between replays: clear the outputs, count another batch
        # with the same workspace, synchronise
        out.fill_(-1)
        status.fill_(-9)
        og, _ = P.count_batch(oplan, workspace=ws)
        torch.cuda.synchronize()
        print(f"[gpu] replay {rep}", flush=True)
        graph.replay()
        torch.cuda.synchronize()
        assert int(status.item()) == 0, rep
        np.testing.assert_array_equal(out.cpu().numpy().view(np.uint64), want, err_msg=f"replay {rep}")
    del graph


def _union_with_cross_edge(b):
    """The union CSR with one extra edge joining graph 0 and graph 1."""
    u = b.union
    uv = u.edges()
    a, c = int(b.node_ptr[0]), int(b.node_ptr[1])
    uv = np.concatenate([uv, np.array([[a, c]], dtype=np.int64)])
    rp, col = G.csr_from_edges(u.n, uv[:, 0], uv[:, 1])
    return G.Graph(rp, col, u.types, u.L, "cross")


def test_async_batch_errors():
    import torch

    import paper_2010_14058_amd as P

    b = G.batch_graphs(30, seed=5)
    dev = torch.device("cuda:0")
    # an edge joining two graphs
    x = _union_with_cross_edge(b)
    plan = P.BatchPlan(torch.from_numpy(x.row_ptr).to(dev), torch.from_numpy(x.col).to(dev),
                       torch.from_numpy(x.types).to(dev), b.node_ptr, b.L)
    ws, out, status = _buffers(plan)
    P.count_batch_async(plan, out, status, ws, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert int(status.item()) == 9  # TG_E_BATCH
    # a declared bound below the largest graph
    plan = _plan(b)
    ws, out, status = _buffers(plan)
    P.count_batch_async(plan, out, status, ws, torch.cuda.current_stream(),
                        max_graph_nodes=plan.max_graph_nodes - 1)
    torch.cuda.synchronize()
    assert int(status.item()) == 9
    # an unsorted row
    u = b.union
    col = u.col.copy()
    r0 = int(np.argmax(np.diff(u.row_ptr) >= 2))
    s0 = int(u.row_ptr[r0])
    col[s0], col[s0 + 1] = col[s0 + 1], col[s0]
    plan = P.BatchPlan(torch.from_numpy(u.row_ptr).to(dev), torch.from_numpy(col).to(dev),
                       torch.from_numpy(u.types).to(dev), b.node_ptr, b.L)
    ws, out, status = _buffers(plan)
    P.count_batch_async(plan, out, status, ws, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert int(status.item()) == 2  # TG_E_NOT_SIMPLE
    # the same batch then counts normally with the same buffers
    plan = _plan(b)
    P.count_batch_async(plan, out, status, ws, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert int(status.item()) == 0
