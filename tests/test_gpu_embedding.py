"""GPU parity of the typed-graphlet embeddings (Alg. 5) against the oracle.

* Edge weights W (instances of a typed graphlet containing each edge): bit
  for bit against the oracle's, for every graphlet and type multiset.
* Spectra and embeddings: eigenvalues against the oracle's dense float64
  eigen-decomposition, the eigenvector subspace through its projector U U^T
  (unique whenever the wanted eigenvalues are separated from the next one),
  and the embedding rows through Z Z^T, for every graphlet where the cut
  falls in a gap.

Tolerances.  The solver stops at residual norms ||M x - theta x|| <= tol
(tests: 1e-12), M = (S + I) / 2.  A Ritz value is then within tol^2 / gap
of an eigenvalue and the subspace within sin(angle) <= tol / gap of the
true one, both far below float64 rounding of the products (~1e-13 for
these sizes); the tests allow 1e-9 on eigenvalues of L and 1e-7 on the
projector for cuts with a gap of at least 1e-3.
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
    Z, ev, its = P.graphlet_embedding(rp, col, w, dim, tol=TOL, **kw)
    torch.cuda.synchronize()
    return Z.cpu().numpy(), ev.cpu().numpy(), its


def _check_embedding(oracle_mod, g, rp, col, w, dim, label):
    vals, vecs, act = oracle_mod.laplacian_spectrum(g, w)
    a = int(act.sum())
    k = min(dim, a)
    print(f"[gpu] embedding {label} dim={dim} active={a}", flush=True)
    U, ev, its = _embed(rp, col, w, dim, raw=True)
    Z, ev2, _ = _embed(rp, col, w, dim)
    np.testing.assert_array_equal(ev, ev2)
    np.testing.assert_allclose(ev[:k], vals[:k], rtol=0, atol=1e-9, err_msg=label)
    assert np.all(ev[k:] == 0) and np.all(U[:, k:] == 0) and np.all(Z[:, k:] == 0)
    assert np.all(U[~act] == 0) and np.all(Z[~act] == 0)
    # orthonormal columns
    np.testing.assert_allclose(U[:, :k].T @ U[:, :k], np.eye(k), rtol=0, atol=1e-10)
    # Alg. 5's rows: unit length where the eigenvector rows are nonzero
    nrm = np.sqrt((Z * Z).sum(axis=1))
    rown = np.sqrt((U * U).sum(axis=1))
    np.testing.assert_allclose(nrm[rown > 0], 1.0, rtol=0, atol=1e-12)
    gap = vals[k] - vals[k - 1] if k < a else np.inf
    if gap < 1e-3:
        return False
    Uo = np.zeros((g.n, k))
    Uo[act] = vecs[:, :k]
    Po, Pg = Uo @ Uo.T, U[:, :k] @ U[:, :k].T
    np.testing.assert_allclose(Pg, Po, rtol=0, atol=1e-7, err_msg=label)
    if g.n > 1000:
        return True
    # rows of the embedding: Z Z^T on rows whose eigenvector rows are not tiny
    _, Zo = oracle_mod.embedding(g, w, dim)
    big = (Uo * Uo).sum(axis=1) > 1e-4
    np.testing.assert_allclose((Z @ Z.T)[np.ix_(big, big)], (Zo @ Zo.T)[np.ix_(big, big)],
                               rtol=0, atol=1e-5, err_msg=label)
    return True


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
    assert checked >= 60


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
    """Two Gram and residual chunks (2048 rows each) with a ragged tail."""
    g = planted_partition(2600, 5, 12.0, 0.5, 9)
    rp, col, ty, rows, uv = _device_graph(g)
    orows = oracle_mod.all_edge_rows(g)
    for h, ms in ((0, (0, 0)), (1, (0, 0, 0))):
        w = oracle_mod.graphlet_edge_weights(g, orows, h, ms)
        assert _check_embedding(oracle_mod, g, rp, col, w, 5, f"{g.name} h{h}")


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
    # triangles only: 3 active nodes, fewer than dim -> spectrum {0, 1.5, 1.5}
    w = oracle_mod.graphlet_edge_weights(g, orows, 2, (0, 0, 0))
    U, ev, its = _embed(rp, col, w, 6, raw=True)
    np.testing.assert_allclose(ev[:3], [0.0, 1.5, 1.5], atol=1e-12)
    assert np.all(ev[3:] == 0) and np.all(U[:, 3:] == 0) and np.all(U[3:] == 0)
    # edges: two components -> eigenvalue 0 twice; node 8 isolated, zero row
    w = oracle_mod.graphlet_edge_weights(g, orows, 0, (0, 0))
    Z, ev, its = _embed(rp, col, w, 2)
    np.testing.assert_allclose(ev, [0.0, 0.0], atol=1e-12)
    assert np.all(Z[8] == 0)
    # no instance (4-cliques): zero rows and eigenvalues, no iteration
    w = oracle_mod.graphlet_edge_weights(g, orows, 8, (0, 0, 0, 0))
    assert not w.any()
    Z, ev, its = _embed(rp, col, w, 4)
    assert its == 0 and not Z.any() and not ev.any()
    # no edges at all
    e0 = G.Graph(np.zeros(5, dtype=np.int64), np.zeros(0, dtype=np.int32),
                 np.zeros(4, dtype=np.uint8), 1, "empty")
    rp0, col0, _ = to_device(e0)
    Z, ev, its = P.graphlet_embedding(rp0, col0, torch.zeros(0, dtype=torch.int64,
                                                             device=device()), 3)
    assert its == 0 and not Z.cpu().numpy().any()


def test_embedding_deterministic_and_seed_free(oracle_mod):
    g = G.chung_lu_typed(800, 8.0, 2.3, 60.0, 2, seed=21, name="cl800")
    rp, col, ty, rows, uv = _device_graph(g)
    w = _gpu_weights(g, rows, uv, ty, 3, (0, 0, 1, 1))
    a = _embed(rp, col, w, 8, seed=1)
    b = _embed(rp, col, w, 8, seed=1)
    c = _embed(rp, col, w, 8, seed=2)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
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
    import paper_2010_14058_amd as P

    g = G.chung_lu_typed(3000, 6.0, 2.2, 80.0, 1, seed=4, name="cl3000")
    rp, col, ty, rows, uv = _device_graph(g)
    w = _gpu_weights(g, rows, uv, ty, 0, (0, 0))
    import torch

    wd = torch.from_numpy(w.view(np.int64).copy()).to(device())
    with pytest.raises(P.TGError) as ei:
        P.graphlet_embedding(rp, col, wd, 16, max_iter=1, degree=2, tol=1e-14)
    assert ei.value.code == P.NO_CONVERGENCE
    Z, ev, its = P.graphlet_embedding(rp, col, wd, 16, max_iter=1, degree=2, tol=1e-14,
                                      check=False)
    assert its == 1
