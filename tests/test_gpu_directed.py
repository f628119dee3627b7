"""GPU parity of the directed typed graphlet counts (Sec. 4.8) against the
oracle, bit for bit: per-edge rows and global counts per canonical class,
on hand-worked digraphs, random small typed digraphs (every mix of single
and reciprocal arcs, L = 1..5), the Erdos-Renyi configuration in full, a
power-law graph with hubs, L = 16 (global counts beyond the LDS histogram),
empty and edgeless inputs, input errors, and the 1M-node power-law
configuration (sampled edges against the oracle; every edge against the
undirected rows the direction splits must add up to)."""

from __future__ import annotations

import numpy as np
import pytest

from gpu_util import device, to_device
from tg_synth import graphs as G

pytestmark = pytest.mark.gpu


def run_directed(g, dirs, per_edge=True):
    import torch

    import paper_2010_14058_amd as P

    print(f"[gpu] directed {g.name}: n={g.n} m={g.m} L={g.L}", flush=True)
    rp, col, ty = to_device(g)
    d = torch.from_numpy(np.ascontiguousarray(dirs)).to(device())
    rows, glob = P.count_directed(rp, col, d, ty, g.L, per_edge=per_edge)
    torch.cuda.synchronize()
    r = rows.cpu().numpy().view(np.uint64) if rows is not None else None
    return r, glob.cpu().numpy().view(np.uint64)


def check(oracle_mod, g, dirs, brute=False):
    D = oracle_mod.directed
    rows, glob = run_directed(g, dirs)
    want = D.edge_rows(g, dirs)
    np.testing.assert_array_equal(rows, want, err_msg=g.name)
    wg = D.global_brute_force(g, dirs) if brute else D.global_from_rows(g, dirs, want)
    np.testing.assert_array_equal(glob, wg, err_msg=g.name)
    _, glob2 = run_directed(g, dirs, per_edge=False)
    np.testing.assert_array_equal(glob2, glob)


def _hand(n, arcs, types, L):
    und = sorted({tuple(sorted(a)) for a in arcs})
    e = np.asarray(und, dtype=np.int64).reshape(-1, 2)
    rp, col = G.csr_from_edges(n, e[:, 0], e[:, 1])
    g = G.Graph(rp, col, np.asarray(types, dtype=np.uint8), L, "hand")
    s = set(arcs)
    dirs = np.zeros(g.nnz, dtype=np.uint8)
    for u in range(n):
        for q in range(int(rp[u]), int(rp[u + 1])):
            x = int(col[q])
            dirs[q] = (1 if (u, x) in s else 0) | (2 if (x, u) in s else 0)
    return g, dirs


def test_hand_digraphs(oracle_mod):
    cases = [(3, [(0, 1), (1, 2), (2, 0)], [0, 0, 0], 1),
             (3, [(0, 1), (0, 2), (1, 2)], [0, 0, 0], 1),
             (3, [(0, 1), (1, 0), (1, 2)], [0, 1, 0], 2),
             (5, [(0, 1), (1, 0), (0, 2), (2, 0), (1, 2), (2, 1), (3, 0), (1, 4), (4, 3)],
              [0, 1, 1, 0, 2], 3)]
    for n, arcs, types, L in cases:
        g, dirs = _hand(n, arcs, types, L)
        check(oracle_mod, g, dirs, brute=True)


def test_random_small(oracle_mod):
    rng = np.random.default_rng(31)
    for s in range(40):
        n = int(rng.integers(3, 40))
        L = int(rng.integers(1, 6))
        g = G.random_small_graph(n, float(rng.uniform(0.05, 0.9)), L, 900 + s)
        dirs = G.orient(g, float(rng.choice([0.0, 0.3, 1.0])), s)
        check(oracle_mod, g, dirs, brute=n <= 14)


def test_er_config_full(oracle_mod):
    g = G.config_graph(1, seed=0)
    check(oracle_mod, g, G.orient(g, 0.2, 1))


def test_power_law_hubs(oracle_mod):
    g = G.chung_lu_typed(3000, 10.0, 2.1, 600.0, 4, seed=5, name="cl3000_hubs")
    assert int(g.degrees().max()) > 200
    check(oracle_mod, g, G.orient(g, 0.1, 2))


def test_sixteen_types(oracle_mod):
    g = G.er_graph(400, 12.0, 16, seed=3, name="er400_L16")
    check(oracle_mod, g, G.orient(g, 0.3, 3))


def test_empty_and_edgeless(oracle_mod):
    g = G.Graph(np.zeros(6, dtype=np.int64), np.zeros(0, dtype=np.int32),
                np.zeros(5, dtype=np.uint8), 2, "edgeless")
    rows, glob = run_directed(g, np.zeros(0, dtype=np.uint8))
    assert rows.shape == (0, 30) and not glob.any()


def test_input_errors():
    import torch

    import paper_2010_14058_amd as P

    g = G.random_small_graph(8, 0.6, 2, 4)
    good = G.orient(g, 0.3, 0)
    rp, col, ty = to_device(g)
    dev = device()
    bad = good.copy()
    bad[0] = 0                                   # a slot without an arc
    with pytest.raises(P.TGError) as ei:
        P.count_directed(rp, col, torch.from_numpy(bad).to(dev), ty, 2)
    assert ei.value.code == 2
    bad = good.copy()
    bad[0] = 3 if good[0] != 3 else 1            # reverse slot no longer mirrored
    with pytest.raises(P.TGError) as ei:
        P.count_directed(rp, col, torch.from_numpy(bad).to(dev), ty, 2)
    assert ei.value.code == 2
    tyb = ty.clone()
    tyb[0] = 5                                   # type >= L
    with pytest.raises(P.TGError) as ei:
        P.count_directed(rp, col, torch.from_numpy(good).to(dev), tyb, 2)
    assert ei.value.code == 3


def test_power_law_1m_sampled(oracle_mod):
    """The 1M-node, 10M-edge Chung-Lu configuration with 20% reciprocal
    edges: 3,000 sampled edges (and every hub edge among them) against the
    oracle; every edge's direction splits against the undirected rows; the
    global classes against the undirected global counts."""
    import torch

    import paper_2010_14058_amd as P

    D = oracle_mod.directed
    g = G.config_graph(2, seed=0)
    dirs = G.orient(g, 0.2, 7)
    rows, glob = run_directed(g, dirs)
    rp, col, ty = to_device(g)
    urows, uglob = P.count_typed_graphlets(rp, col, ty, g.L)
    torch.cuda.synchronize()
    urows = urows.cpu().numpy().view(np.uint64)
    uglob = uglob.cpu().numpy().view(np.uint64)
    L = g.L
    uv = g.edges()
    rng = np.random.default_rng(0)
    deg = g.degrees()
    hub = np.flatnonzero(np.maximum(deg[uv[:, 0]], deg[uv[:, 1]]) > 5000)
    sample = np.unique(np.concatenate([rng.choice(g.m, 3000, replace=False),
                                       rng.choice(hub, min(200, hub.size), replace=False)]))
    for e in sample.tolist():
        i, j = uv[e]
        np.testing.assert_array_equal(rows[e], D.edge_row(g, dirs, int(i), int(j)),
                                      err_msg=f"edge {e} ({i},{j})")
    # direction splits add up to the undirected typed rows (tri first, then path3)
    tri = rows[:, :9 * L].reshape(-1, L, 9).sum(axis=2)
    path = rows[:, 9 * L:12 * L].reshape(-1, L, 3).sum(axis=2) + \
        rows[:, 12 * L:].reshape(-1, L, 3).sum(axis=2)
    np.testing.assert_array_equal(tri, urows[:, :L])
    np.testing.assert_array_equal(path, urows[:, L:2 * L])
    # global: 2-node classes sum to the edges; 3-node triangles and paths to
    # the undirected instance totals
    assert int(glob[:4 * L * L].sum()) == g.m
    body = glob[4 * L * L:].reshape(-1, 64)
    codes = np.arange(64)
    nedges = (codes >> 4 > 0).astype(int) + ((codes >> 2) & 3 > 0) + ((codes & 3) > 0)
    ntri_dir = int(body[:, nedges == 3].sum())
    npath_dir = int(body[:, nedges == 2].sum())
    from math import comb

    n2 = comb(L + 1, 2)           # undirected layout: h0, then h1 (3-paths), h2 (triangles)
    n3 = comb(L + 2, 3)
    assert ntri_dir == int(uglob[n2 + n3:n2 + 2 * n3].sum())
    assert npath_dir == int(uglob[n2:n2 + n3].sum())
