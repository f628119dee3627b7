"""Batched counting: many graphs in one call must give, for every graph,
exactly the counts of the oracle (and of the single-graph entry point)."""

import numpy as np
import pytest

import brute_force as BF
from tg_synth import graphs as G

pytestmark = pytest.mark.gpu


def _plan(b):
    import torch

    import paper_2010_14058_amd as P

    dev = torch.device("cuda:0")
    u = b.union
    return P.BatchPlan(torch.from_numpy(u.row_ptr).to(dev), torch.from_numpy(u.col).to(dev),
                       torch.from_numpy(u.types).to(dev), b.node_ptr, b.L)


def _expand(row, Lg, Lmax):
    """Oracle row in the Lg layout -> the Lmax layout."""
    src, dst = BF.column_index(Lg), BF.column_index(Lmax)
    out = np.zeros(len(dst), dtype=np.uint64)
    for name, c in src.items():
        out[dst[name]] = row[c]
    return out


def test_batch_against_oracle(oracle_mod):
    import torch

    import paper_2010_14058_amd as P

    b = G.batch_graphs(400, seed=3)
    print(f"[gpu] batch of {b.G} graphs, n={b.union.n} m={b.union.m}", flush=True)
    plan = _plan(b)
    glob, rows = P.count_batch(plan, per_edge=True)
    torch.cuda.synchronize()
    glob = glob.cpu().numpy().view(np.uint64)
    rows = rows.cpu().numpy().view(np.uint64)
    ep = b.edge_ptr()
    for g in range(b.G):
        gg = b.graph(g)
        want_rows = oracle_mod.all_edge_rows(gg, threads=4)
        want_glob = oracle_mod.global_counts(gg, want_rows)
        got = glob[plan.goff_host[g]:plan.goff_host[g + 1]]
        np.testing.assert_array_equal(got, want_glob, err_msg=f"graph {g}")
        if g % 20 == 0:
            exp = np.stack([_expand(r, gg.L, b.union.L) for r in want_rows]) if gg.m else \
                np.zeros((0, rows.shape[1]), np.uint64)
            np.testing.assert_array_equal(rows[ep[g]:ep[g + 1]], exp, err_msg=f"rows of graph {g}")


def test_batch_equals_single_calls():
    import torch

    import paper_2010_14058_amd as P
    from gpu_util import run_gpu

    b = G.batch_graphs(60, seed=9)
    plan = _plan(b)
    glob, _ = P.count_batch(plan)
    torch.cuda.synchronize()
    glob = glob.cpu().numpy().view(np.uint64)
    for g in range(b.G):
        _, single = run_gpu(b.graph(g))
        np.testing.assert_array_equal(glob[plan.goff_host[g]:plan.goff_host[g + 1]], single)


def test_batch_with_hubs_and_max_L(oracle_mod):
    """A batch mixing a power-law graph with hubs (heavy paths) and L = 16."""
    import torch

    import paper_2010_14058_amd as P

    parts = [G.chung_lu_typed(3000, 12.0, 2.1, 1500.0, 16, seed=4),
             G.random_small_graph(12, 0.5, 3, 77),
             G.chung_lu_typed(500, 8.0, 2.1, 60.0, 2, seed=8)]
    offs = np.cumsum([0] + [p.n for p in parts])
    rp = [np.zeros(1, np.int64)]
    cols, types = [], []
    base = 0
    for p, o in zip(parts, offs[:-1]):
        rp.append(p.row_ptr[1:] + base)
        base += p.nnz
        cols.append(p.col + o)
        types.append(p.types)
    u = G.Graph(np.concatenate(rp), np.concatenate(cols).astype(np.int32),
                np.concatenate(types), 16, "mix")
    b = G.GraphBatch(u, offs.astype(np.int64), np.array([p.L for p in parts], np.int32))
    plan = _plan(b)
    glob, _ = P.count_batch(plan)
    torch.cuda.synchronize()
    glob = glob.cpu().numpy().view(np.uint64)
    for g, p in enumerate(parts):
        want = oracle_mod.global_counts(p, oracle_mod.all_edge_rows(p, threads=8))
        np.testing.assert_array_equal(glob[plan.goff_host[g]:plan.goff_host[g + 1]], want)


def _batch_status(row_ptr, col, types, node_ptr, graph_L):
    import torch

    import paper_2010_14058_amd as P

    dev = torch.device("cuda:0")
    plan = P.BatchPlan(torch.from_numpy(np.asarray(row_ptr, np.int64)).to(dev),
                       torch.from_numpy(np.asarray(col, np.int32)).to(dev),
                       torch.from_numpy(np.asarray(types, np.uint8)).to(dev), node_ptr, graph_L)
    try:
        P.count_batch(plan)
        torch.cuda.synchronize()
    except P.TGError as e:
        return e.code
    return 0


def test_batch_invalid_inputs():
    # two graphs: nodes {0,1} and {2,3}; edges 0-1 and 2-3
    rp, col = [0, 1, 2, 3, 4], [1, 0, 3, 2]
    assert _batch_status(rp, col, [0, 1, 0, 1], [0, 2, 4], [2, 2]) == 0
    # an edge between the graphs (1-2 instead of 2-3)
    assert _batch_status([0, 1, 3, 4, 4], [1, 0, 2, 1], [0, 1, 0, 1], [0, 2, 4], [2, 2]) == 9
    # node ranges that do not cover the nodes
    assert _batch_status(rp, col, [0, 1, 0, 1], [0, 2, 3], [2, 2]) == 9
    # a type outside its graph's range (graph 1 has L = 1)
    assert _batch_status(rp, col, [0, 1, 0, 1], [0, 2, 4], [2, 1]) == 3


def _union(parts, L_max):
    offs = np.cumsum([0] + [p.n for p in parts])
    rp = [np.zeros(1, np.int64)]
    cols, types = [], []
    base = 0
    for p, o in zip(parts, offs[:-1]):
        rp.append(p.row_ptr[1:] + base)
        base += p.nnz
        cols.append(p.col + o)
        types.append(p.types)
    u = G.Graph(np.concatenate(rp), np.concatenate(cols).astype(np.int32),
                np.concatenate(types), L_max, "mix")
    return G.GraphBatch(u, offs.astype(np.int64), np.array([p.L for p in parts], np.int32))


def test_batch_with_degree_above_16_bits():
    """A batch whose first graph has a node of degree 70000: the batch is
    relabelled graph by graph (node ids not ranked by degree), so every
    4-cycle map entry takes 32-bit counts, with every group sent to the
    heavy path; each graph's vector equals its single-graph call."""
    import torch

    import paper_2010_14058_amd as P
    from gpu_util import run_gpu

    rng = np.random.default_rng(13)
    leaves = 70_000
    n = leaves + 2
    a = [np.zeros(leaves, np.int64), np.full(leaves // 4, 1, np.int64)]
    b = [np.arange(2, n, dtype=np.int64), rng.choice(np.arange(2, n), leaves // 4, replace=False)]
    extra = rng.integers(2, n, size=(60_000, 2))
    extra = extra[extra[:, 0] != extra[:, 1]]
    u = np.concatenate(a + [extra[:, 0], np.array([0])])
    v = np.concatenate(b + [extra[:, 1], np.array([1])])
    e = np.unique(np.sort(np.stack([u, v], 1), axis=1), axis=0)
    rp, col = G.csr_from_edges(n, e[:, 0], e[:, 1])
    hub = G.Graph(rp, col, rng.integers(0, 3, size=n).astype(np.uint8), 3, "hub70k_batch")
    assert hub.degrees().max() > 65535
    parts = [hub, G.random_small_graph(15, 0.4, 3, 5), G.chung_lu_typed(800, 8.0, 2.1, 90.0, 3,
                                                                        seed=6)]
    bt = _union(parts, 3)
    old = P.set_tuning(light_wedges=1)
    try:
        print(f"[gpu] batch with a 70k hub: n={bt.union.n} m={bt.union.m}", flush=True)
        plan = _plan(bt)
        glob, _ = P.count_batch(plan)
        torch.cuda.synchronize()
        glob = glob.cpu().numpy().view(np.uint64)
        assert P.last_stats()["heavy_groups"] > 0
        for g, p in enumerate(parts):
            _, single = run_gpu(p, per_edge=False)
            np.testing.assert_array_equal(glob[plan.goff_host[g]:plan.goff_host[g + 1]], single)
    finally:
        P.set_tuning(**old)
