"""GPU parity of the typed-graphlet embeddings (Alg. 5) against the oracle.

* Edge weights W (instances of a typed graphlet containing each edge): bit
  for bit against the oracle's, for every graphlet and type multiset.
* Components of the typed-graphlet graph G^H (Sec. 8.8 embeds each one on
  its own): component ids bit for bit.
* Spectra and embeddings, per component: eigenvalues against the oracle's
  dense float64 eigen-decomposition, the eigenvector subspace through its
  projector U U^T (unique whenever the wanted eigenvalues are separated
  from the next one, or the component has at most dim nodes), and the
  embedding rows through Z Z^T.  Components of at most 64 nodes go through
  the dense Jacobi kernel, larger ones through the filtered subspace
  iteration; the cases cover both, several Gram chunks, and blocks as wide
  as the component.

Tolerances.  The subspace iteration stops at residual norms ||M x - theta
x|| <= tol (tests: 1e-12), M = (S + I) / 2.  A Ritz value is then within
tol^2 / gap of an eigenvalue and the subspace within sin(angle) <= tol /
gap of the true one, both far below float64 rounding of the products
(~1e-13 here); the dense solver is accurate to rounding.  The tests allow
1e-9 on eigenvalues of L and 1e-7 on projectors of components whose cut
has a gap of at least 1e-3.
"""

from __future__ import annotations

import numpy as np
import pytest

import brute_force as BF
from gpu_util import device, to_device
from tg_synth import graphs as G

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _multisets(L, h):
    return BF.multisets(L, 2 if h == 0 else 3 if h <= 2 else 4)


def _gpu_weights(g, rows_dev, uv_dev, ty_dev, h, ms):
    import paper_2010_14058_amd as P

    w = P.graphlet_weights(rows_dev, uv_dev, ty_dev, g.L, h, ms)
    return w.cpu().numpy().view(np.uint64)


def _device_graph(g):
    import torch

    import paper_2010_14058_amd as P

    rp, col, ty = to_device(g)
    rows, _ = P.count_typed_graphlets(rp, col, ty, g.L)
    uv = P.edge_list(rp, col)
    torch.cuda.synchronize()
    return rp, col, ty, rows, uv


def _embed(rp, col, w_np, dim, **kw):
    import torch

    import paper_2010_14058_amd as P

    w = torch.from_numpy(w_np.view(np.int64).copy()).to(device())
    Z, ev, comp, its = P.graphlet_embedding(rp, col, w, dim, tol=TOL, **kw)
    torch.cuda.synchronize()
    return Z.cpu().numpy(), ev.cpu().numpy(), comp.cpu().numpy(), its


def _check_embedding(oracle_mod, g, rp, col, w, dim, label):
    """Checks one embedding against the oracle; returns the number of
    components whose subspace is unique (and so was compared)."""
    ev_o, U_o, comp_o = oracle_mod.embedding(g, w, dim, raw=True)
    print(f"[gpu] embedding {label} dim={dim} components={len(np.unique(comp_o[comp_o >= 0]))}",
          flush=True)
    U, ev, comp, its = _embed(rp, col, w, dim, raw=True)
    Z, ev2, comp2, _ = _embed(rp, col, w, dim)
    np.testing.assert_array_equal(comp, comp_o, err_msg=label)
    np.testing.assert_array_equal(comp2, comp_o)
    np.testing.assert_array_equal(ev, ev2)
    np.testing.assert_allclose(ev, ev_o, rtol=0, atol=1e-9, err_msg=label)
    out = comp < 0
    assert not U[out].any() and not Z[out].any()
    nrm = np.sqrt((Z * Z).sum(axis=1))
    np.testing.assert_allclose(nrm[~out], 1.0, rtol=0, atol=1e-12)
    Zo = None
    unique = 0
    for r in np.unique(comp_o[comp_o >= 0]):
        nodes = np.flatnonzero(comp_o == r)
        s = nodes.shape[0]
        k = min(dim, s)
        Uc, Uoc = U[nodes, :k], U_o[nodes, :k]
        assert not U[nodes, k:].any() and not Z[nodes, k:].any()
        np.testing.assert_allclose(Uc.T @ Uc, np.eye(k), rtol=0, atol=1e-10, err_msg=label)
        if k < s:
            vals, _, _ = oracle_mod.laplacian_spectrum(g, w, nodes)
            if vals[k] - vals[k - 1] < 1e-3:
                continue
        unique += 1
        np.testing.assert_allclose(Uc @ Uc.T, Uoc @ Uoc.T, rtol=0, atol=1e-7,
                                   err_msg=f"{label} component {r}")
        if g.n <= 1000:
            if Zo is None:
                _, Zo, _ = oracle_mod.embedding(g, w, dim)
            big = nodes[(Uoc * Uoc).sum(axis=1) > 1e-4]
            np.testing.assert_allclose(Z[big] @ Z[big].T, Zo[big] @ Zo[big].T, rtol=0, atol=1e-5,
                                       err_msg=f"{label} component {r}")
    return unique


def test_weights_all_graphlets(oracle_mod):
    graphs = [G.chung_lu_typed(500, 8.0, 2.3, 60.0, 3, seed=11, name="cl500_L3"),
              G.er_graph(300, 10.0, 2, seed=5, name="er300_L2"),
              G.random_small_graph(12, 0.7, 3, 41),
              G.chung_lu_typed(400, 6.0, 2.1, 80.0, 1, seed=2, name="cl400_L1")]
    for g in graphs:
        rp, col, ty, rows, uv = _device_graph(g)
        orows = oracle_mod.all_edge_rows(g)
        np.testing.assert_array_equal(uv.cpu().numpy(), g.edges())
        print(f"[gpu] weights {g.name} m={g.m}", flush=True)
        for h in range(9):
            for ms in _multisets(g.L, h):
                want = oracle_mod.graphlet_edge_weights(g, orows, h, ms)
                got = _gpu_weights(g, rows, uv, ty, h, ms)
                np.testing.assert_array_equal(got, want, err_msg=f"{g.name} h{h} {ms}")


def test_embedding_every_graphlet(oracle_mod):
    g = G.chung_lu_typed(600, 8.0, 2.3, 60.0, 2, seed=3, name="cl600_L2")
    rp, col, ty, rows, uv = _device_graph(g)
    orows = oracle_mod.all_edge_rows(g)
    checked = 0
    for h in range(9):
        for ms in _multisets(g.L, h):
            w = oracle_mod.graphlet_edge_weights(g, orows, h, ms)
            for dim in (1, 4, 16):
                checked += _check_embedding(oracle_mod, g, rp, col, w, dim, f"h{h} {ms}")
    assert checked >= 100


def planted_partition(n, k, d_in, d_out, seed):
    """k equal blocks, about d_in neighbours inside a node's block and d_out
    outside it: k small Laplacian eigenvalues, then a wide gap."""
    rng = np.random.default_rng(seed)
    blk = np.arange(n) * k // n
    iu, ju = np.triu_indices(n, 1)
    p = np.where(blk[iu] == blk[ju], d_in / (n / k), d_out / n)
    pick = rng.random(iu.shape[0]) < p
    rp, col = G.csr_from_edges(n, iu[pick], ju[pick])
    return G.Graph(rp, col, np.zeros(n, dtype=np.uint8), 1, f"planted_n{n}_k{k}")


def test_embedding_multi_chunk(oracle_mod):
    """A component of 2,600 nodes: two Gram and residual chunks (2048 rows
    each) with a ragged tail."""
    g = planted_partition(2600, 5, 12.0, 0.5, 9)
    rp, col, ty, rows, uv = _device_graph(g)
    orows = oracle_mod.all_edge_rows(g)
    for h, ms in ((0, (0, 0)), (1, (0, 0, 0))):
        w = oracle_mod.graphlet_edge_weights(g, orows, h, ms)
        assert _check_embedding(oracle_mod, g, rp, col, w, 5, f"{g.name} h{h}") >= 1


def many_components(sizes, avg_degree, seed):
    """Disjoint G(s, p) pieces of the given sizes (each may split further),
    node ids shuffled so that components interleave."""
    rng = np.random.default_rng(seed)
    n = int(sum(sizes))
    perm = rng.permutation(n)
    us, vs, base = [], [], 0
    for s in sizes:
        iu, ju = np.triu_indices(s, 1)
        pick = rng.random(iu.shape[0]) < min(1.0, avg_degree / max(s - 1, 1))
        us.append(perm[base + iu[pick]])
        vs.append(perm[base + ju[pick]])
        base += s
    u, v = np.concatenate(us), np.concatenate(vs)
    rp, col = G.csr_from_edges(n, np.minimum(u, v), np.maximum(u, v))
    types = rng.integers(0, 2, n).astype(np.uint8)
    return G.Graph(rp, col, types, 2, f"pieces_{len(sizes)}_s{seed}")


def test_embedding_many_components(oracle_mod):
    """Dozens of components from 2 to 300 nodes: the dense kernel (<= 64
    nodes) and the subspace iteration, with blocks narrower than, as wide
    as, and capped by the component."""
    sizes = [2, 3, 4, 5, 7, 9, 12, 16, 20, 30, 40, 50, 63, 64, 65, 66, 70, 80, 90, 100, 150, 300]
    g = many_components(sizes * 2, 5.0, 17)
    rp, col, ty, rows, uv = _device_graph(g)
    orows = oracle_mod.all_edge_rows(g)
    checked = 0
    for h, ms in ((0, (0, 1)), (0, (0, 0)), (1, (0, 0, 1)), (3, (0, 0, 1, 1))):
        w = oracle_mod.graphlet_edge_weights(g, orows, h, ms)
        for dim in (3, 16, 64):
            checked += _check_embedding(oracle_mod, g, rp, col, w, dim, f"{g.name} h{h} {ms}")
    assert checked >= 200
    # blocks wider than the LDS-resident solvers take (p > 192)
    w = oracle_mod.graphlet_edge_weights(g, orows, 3, (0, 0, 1, 1))
    assert _check_embedding(oracle_mod, g, rp, col, w, 200, f"{g.name} wide") >= 30


def test_embedding_clustered_spectrum():
    """Weights given directly: a 10-node weighted cycle with 40 pendant
    pairs c - a - b, W(c, a) = 1 and W(a, b) = 1000 + 7k.  Each pair adds
    an eigenvalue near 1 / (2 W(a, b)), so 39 eigenvalues within 5e-4 of
    each other follow the zero eigenvalue and the cut at dim = 16 falls
    inside that cluster: the block must widen to hold the cluster before
    the wanted residuals can fall.  Checked against a dense eigensolve of
    the same Laplacian: eigenvalues, orthonormality and residuals (the
    subspace inside the cluster is not unique)."""
    import torch

    import paper_2010_14058_amd as P

    core = 10
    edges, wts = [], []
    for i in range(core):
        edges.append((i, (i + 1) % core))
        wts.append(1)
    nxt = core
    for k in range(40):
        c, a, b = k % core, nxt, nxt + 1
        nxt += 2
        edges += [(c, a), (a, b)]
        wts += [1, 1000 + 7 * k]
    n = nxt
    e = np.array([tuple(sorted(x)) for x in edges])
    order = np.lexsort((e[:, 1], e[:, 0]))
    e, wv = e[order], np.array(wts, dtype=np.uint64)[order]
    rp_np, col_np = G.csr_from_edges(n, e[:, 0], e[:, 1])
    g = G.Graph(rp_np, col_np, np.zeros(n, dtype=np.uint8), 1, "clustered")
    np.testing.assert_array_equal(g.edges(), e)
    Wd = np.zeros((n, n))
    Wd[e[:, 0], e[:, 1]] = wv
    Wd[e[:, 1], e[:, 0]] = wv
    d = Wd.sum(axis=1)
    Lap = np.eye(n) - Wd / np.sqrt(np.outer(d, d))
    vals = np.linalg.eigvalsh(Lap)
    assert vals[39] - vals[1] < 1e-3 and vals[40] - vals[39] > 0.5    # the cluster
    rp, col, _ = to_device(g)
    dim = 16
    U, ev, comp, its = _embed(rp, col, wv, dim, raw=True)
    print(f"[gpu] clustered spectrum: {its} iterations", flush=True)
    assert its > 25                       # the first block stalled
    assert np.all(comp == 0)
    np.testing.assert_allclose(ev[0], vals[:dim], rtol=0, atol=1e-9)
    np.testing.assert_allclose(U.T @ U, np.eye(dim), rtol=0, atol=1e-10)
    res = np.linalg.norm(Lap @ U - U * ev[0][None, :], axis=0)
    assert res.max() < 1e-9


def test_embedding_degenerate_cases(oracle_mod):
    import torch

    import paper_2010_14058_amd as P

    # a triangle and a disjoint 4-cycle with a pendant node, L = 1
    edges = [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (5, 6), (3, 6), (6, 7)]
    e = np.asarray(edges)
    rp_np, col_np = G.csr_from_edges(9, e[:, 0], e[:, 1])
    g = G.Graph(rp_np, col_np, np.zeros(9, dtype=np.uint8), 1, "tri+c4")
    rp, col, ty, rows, uv = _device_graph(g)
    orows = oracle_mod.all_edge_rows(g)
    # triangles only: one component of 3 nodes, fewer than dim
    w = oracle_mod.graphlet_edge_weights(g, orows, 2, (0, 0, 0))
    U, ev, comp, its = _embed(rp, col, w, 6, raw=True)
    np.testing.assert_array_equal(comp, [0, 0, 0] + [-1] * 6)
    np.testing.assert_allclose(ev[0, :3], [0.0, 1.5, 1.5], atol=1e-12)
    assert not ev[0, 3:].any() and not ev[1:].any() and its == 0
    np.testing.assert_allclose(U[:3, :3] @ U[:3, :3].T, np.eye(3), atol=1e-12)
    assert not U[:, 3:].any() and not U[3:].any()
    # edges: two components, each with eigenvalue 0; node 8 in none
    w = oracle_mod.graphlet_edge_weights(g, orows, 0, (0, 0))
    Z, ev, comp, its = _embed(rp, col, w, 2)
    np.testing.assert_array_equal(comp, [0, 0, 0, 3, 3, 3, 3, 3, -1])
    np.testing.assert_allclose(ev[[0, 3], 0], [0.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(ev[0, 1], 1.5, atol=1e-12)
    assert not Z[8].any()
    # no instance (4-cliques): nothing to embed
    w = oracle_mod.graphlet_edge_weights(g, orows, 8, (0, 0, 0, 0))
    assert not w.any()
    Z, ev, comp, its = _embed(rp, col, w, 4)
    assert its == 0 and not Z.any() and not ev.any() and np.all(comp == -1)
    # no edges at all
    e0 = G.Graph(np.zeros(5, dtype=np.int64), np.zeros(0, dtype=np.int32),
                 np.zeros(4, dtype=np.uint8), 1, "empty")
    rp0, col0, _ = to_device(e0)
    Z, ev, comp, its = P.graphlet_embedding(rp0, col0, torch.zeros(0, dtype=torch.int64,
                                                                   device=device()), 3)
    assert its == 0 and not Z.cpu().numpy().any() and np.all(comp.cpu().numpy() == -1)


def test_embedding_deterministic_and_seed_free(oracle_mod):
    g = G.chung_lu_typed(800, 8.0, 2.3, 60.0, 2, seed=21, name="cl800")
    rp, col, ty, rows, uv = _device_graph(g)
    w = _gpu_weights(g, rows, uv, ty, 3, (0, 0, 1, 1))
    a = _embed(rp, col, w, 8, seed=1)
    b = _embed(rp, col, w, 8, seed=1)
    c = _embed(rp, col, w, 8, seed=2)
    assert a[3] > 0           # the giant component went through the iteration
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a[2], c[2])
    np.testing.assert_allclose(a[1], c[1], rtol=0, atol=1e-9)


def test_embedding_input_checks():
    import torch

    import paper_2010_14058_amd as P

    dev = device()
    # asymmetric: 0 -> 1 without 1 -> 0 (and nnz even)
    rp = torch.tensor([0, 2, 2, 2], dtype=torch.int64, device=dev)
    col = torch.tensor([1, 2], dtype=torch.int32, device=dev)
    w = torch.ones(1, dtype=torch.int64, device=dev)
    with pytest.raises(P.TGError):
        P.graphlet_embedding(rp, col, w, 2)
    # unsorted row
    rp = torch.tensor([0, 2, 3, 4], dtype=torch.int64, device=dev)
    col = torch.tensor([2, 1, 0, 0], dtype=torch.int32, device=dev)
    w = torch.ones(2, dtype=torch.int64, device=dev)
    with pytest.raises(P.TGError):
        P.graphlet_embedding(rp, col, w, 2)
    # row pointer not ending at nnz
    rp = torch.tensor([0, 1, 3], dtype=torch.int64, device=dev)
    col = torch.tensor([1, 0], dtype=torch.int32, device=dev)
    with pytest.raises(P.TGError):
        P.graphlet_embedding(rp, col, torch.ones(1, dtype=torch.int64, device=dev), 2)


def test_embedding_iteration_limit():
    """max_iter = 1 on a graph whose spectrum needs more: TG_E_NO_CONVERGENCE
    with check, the last Ritz pairs without."""
    import torch

    import paper_2010_14058_amd as P

    g = G.chung_lu_typed(3000, 6.0, 2.2, 80.0, 1, seed=4, name="cl3000")
    rp, col, ty, rows, uv = _device_graph(g)
    w = _gpu_weights(g, rows, uv, ty, 0, (0, 0))
    wd = torch.from_numpy(w.view(np.int64).copy()).to(device())
    with pytest.raises(P.TGError) as ei:
        P.graphlet_embedding(rp, col, wd, 16, max_iter=1, degree=2, tol=1e-14)
    assert ei.value.code == P.NO_CONVERGENCE
    Z, ev, comp, its = P.graphlet_embedding(rp, col, wd, 16, max_iter=1, degree=2, tol=1e-14,
                                            check=False)
    assert its == 1


def test_embedding_full_size_properties(oracle_mod):
    """The 1M-node, 10M-edge power-law configuration, typed 3-paths {0,0,1}
    (a 649k-node component and a small one) and edges {0,1} (6,160
    components) at D = 16: component ids against scipy's connected
    components of the weighted graph; eigenvalues ascending in [0, 2) with
    0 first; the eigenvectors orthonormal with Laplacian residuals
    ||L u - lambda u|| below 1e-8 (scipy sparse products on the host); the
    small components' spectra and projectors against the oracle's dense
    solve, on a sample of them."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    import torch

    import paper_2010_14058_amd as P

    g = G.config_graph(2, seed=0)
    rp, col, ty, rows, uv = _device_graph(g)
    uvn = uv.cpu().numpy()
    for h, ms in ((1, (0, 0, 1)), (0, (0, 1))):
        w = P.graphlet_weights(rows, uv, ty, g.L, h, ms)
        torch.cuda.synchronize()
        wn = w.cpu().numpy().view(np.uint64)
        print(f"[gpu] full-size embedding h{h} {ms}", flush=True)
        U, ev, comp, its = P.graphlet_embedding(rp, col, w, 16, raw=True, tol=1e-10)
        torch.cuda.synchronize()
        U, ev, comp = U.cpu().numpy(), ev.cpu().numpy(), comp.cpu().numpy()
        keep = wn > 0
        Wm = sp.coo_matrix((wn[keep].astype(np.float64), (uvn[keep, 0], uvn[keep, 1])),
                           shape=(g.n, g.n)).tocsr()
        Wm = Wm + Wm.T
        deg = np.asarray(Wm.sum(axis=1)).ravel()
        act = deg > 0
        nc, lab = connected_components(Wm, directed=False)
        # components: same partition, each named by its smallest node id
        first = np.full(nc, g.n, dtype=np.int64)
        np.minimum.at(first, lab[act], np.flatnonzero(act))
        want = np.where(act, first[lab], -1)
        np.testing.assert_array_equal(comp, want)
        roots, sizes = np.unique(comp[comp >= 0], return_counts=True)
        s = np.where(act, 1.0 / np.sqrt(np.where(act, deg, 1.0)), 0.0)
        Sm = sp.diags(s) @ Wm @ sp.diags(s)
        big = roots[sizes > 64]
        for r in big.tolist():
            nodes = np.flatnonzero(comp == r)
            k = min(16, nodes.size)
            lam = ev[r, :k]
            assert abs(lam[0]) < 1e-9 and np.all(np.diff(lam) >= -1e-12) and lam[-1] < 2
            Uc = U[nodes, :k]
            np.testing.assert_allclose(Uc.T @ Uc, np.eye(k), rtol=0, atol=1e-9)
            Ufull = np.zeros((g.n, k))
            Ufull[nodes] = Uc
            res = np.linalg.norm(Ufull - Sm @ Ufull - Ufull * lam[None, :], axis=0)
            assert res.max() < 1e-8, (r, res.max())
        # a sample of the small components against the oracle's dense solve
        # (each component's induced subgraph, ids renumbered in order)
        small = roots[sizes <= 64]
        rng = np.random.default_rng(1)
        ce = np.where(comp[uvn[:, 0]] == comp[uvn[:, 1]], comp[uvn[:, 0]], -1)
        for r in rng.choice(small, min(100, small.size), replace=False).tolist():
            nodes = np.flatnonzero(comp == r)
            em = ce == r
            loc = np.searchsorted(nodes, uvn[em])
            crp, ccol = G.csr_from_edges(nodes.size, loc[:, 0], loc[:, 1])
            gc = G.Graph(crp, ccol, g.types[nodes], g.L, f"component {r}")
            vals, vecs, _ = oracle_mod.laplacian_spectrum(gc, wn[em])
            k = min(16, nodes.size)
            np.testing.assert_allclose(ev[r, :k], vals[:k], rtol=0, atol=1e-9)
            if k == nodes.size or vals[k] - vals[k - 1] > 1e-3:
                Pg = U[nodes, :k] @ U[nodes, :k].T
                np.testing.assert_allclose(Pg, vecs[:, :k] @ vecs[:, :k].T, rtol=0, atol=1e-7)
