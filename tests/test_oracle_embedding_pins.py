"""Pins of the embedding oracle (Alg. 5).

* The typed-graphlet edge weights W against the template brute force, which
  enumerates every 3- and 4-node subset around each edge and counts the
  instances of the typed graphlet that contain it; and their sum against
  |E(H)| times the brute force's global instance count.
* Closed-form spectra of the normalised Laplacian: cycle (1 - cos(2 pi k / n)),
  path (1 - cos(pi k / (n - 1))), complete graph (0 and n / (n - 1)), star
  (0, 1, 2).
* The smallest eigenvector of a connected weighted graph is proportional to
  the square roots of the weighted degrees; scaling W leaves L unchanged;
  embedding rows have unit length, nodes in no instance keep zero rows.
"""

import itertools
import math

import numpy as np
import pytest

import brute_force as BF
from tg_synth import graphs as G

EDGES_OF = {0: 1, 1: 2, 2: 3, 3: 3, 4: 3, 5: 4, 6: 4, 7: 5, 8: 6}


def _graph(n, edges, types, L):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    rp, col = G.csr_from_edges(n, e[:, 0], e[:, 1])
    return G.Graph(rp, col, np.asarray(types, dtype=np.uint8), L, "hand")


def _bf_weights(g, h, ms):
    """Instances of the typed graphlet (h, sorted multiset ms) containing
    each edge, by enumerating node subsets."""
    uv = [tuple(e) for e in g.edges().tolist()]
    adj = BF.adjacency(g.n, uv)
    ty = [int(t) for t in g.types]
    w = {e: 0 for e in uv}
    ms = tuple(ms)
    if h == 0:
        for e in uv:
            w[e] = int(tuple(sorted((ty[e[0]], ty[e[1]]))) == ms)
    elif h in (1, 2):
        for tri in itertools.combinations(range(g.n), 3):
            es = [(x, y) for x, y in itertools.combinations(tri, 2) if adj[x][y]]
            kind = 2 if len(es) == 3 else 1 if len(es) == 2 else 0
            if kind == h and tuple(sorted(ty[x] for x in tri)) == ms:
                for e in es:
                    w[e] += 1
    else:
        for quad in itertools.combinations(range(g.n), 4):
            if not BF._connected(list(quad), adj):
                continue
            hh, orbits = BF._match(list(quad), adj)
            if hh == h and tuple(sorted(ty[x] for x in quad)) == ms:
                for e in orbits:
                    w[tuple(sorted(e))] += 1
    return np.array([w[e] for e in uv], dtype=np.uint64)


def test_weights_against_brute_force(oracle_mod):
    rng = np.random.default_rng(8)
    checked = 0
    for s in range(40):
        n = int(rng.integers(5, 11))
        L = int(rng.integers(1, 4))
        g = G.random_small_graph(n, float(rng.uniform(0.3, 0.9)), L, 800 + s)
        if g.m == 0:
            continue
        rows = oracle_mod.all_edge_rows(g)
        glob = BF.global_instances(g.n, [tuple(e) for e in g.edges().tolist()], g.types, L)
        n2, n3, n4 = (len(BF.multisets(L, k)) for k in (2, 3, 4))
        starts = [0, n2, n2 + n3] + [n2 + 2 * n3 + q * n4 for q in range(6)]
        for h in range(9):
            k = 2 if h == 0 else 3 if h <= 2 else 4
            for q, ms in enumerate(BF.multisets(L, k)):
                w = oracle_mod.graphlet_edge_weights(g, rows, h, ms)
                np.testing.assert_array_equal(w, _bf_weights(g, h, ms), err_msg=f"h{h} {ms}")
                assert int(w.sum()) == EDGES_OF[h] * int(glob[starts[h] + q])
                checked += int(w.sum() > 0)
    assert checked > 100


def _ones(g):
    return np.ones(g.m, dtype=np.uint64)


def test_closed_form_spectra(oracle_mod):
    n = 12
    cyc = _graph(n, [(i, (i + 1) % n) for i in range(n)], [0] * n, 1)
    vals, _, _ = oracle_mod.laplacian_spectrum(cyc, _ones(cyc))
    want = np.sort(1 - np.cos(2 * np.pi * np.arange(n) / n))
    np.testing.assert_allclose(vals, want, atol=1e-12)
    path = _graph(n, [(i, i + 1) for i in range(n - 1)], [0] * n, 1)
    vals, _, _ = oracle_mod.laplacian_spectrum(path, _ones(path))
    np.testing.assert_allclose(vals, np.sort(1 - np.cos(np.pi * np.arange(n) / (n - 1))),
                               atol=1e-12)
    k = 7
    comp = _graph(k, list(itertools.combinations(range(k), 2)), [0] * k, 1)
    vals, _, _ = oracle_mod.laplacian_spectrum(comp, _ones(comp))
    np.testing.assert_allclose(vals, [0.0] + [k / (k - 1)] * (k - 1), atol=1e-12)
    star = _graph(9, [(0, i) for i in range(1, 9)], [0] * 9, 1)
    vals, _, _ = oracle_mod.laplacian_spectrum(star, _ones(star))
    np.testing.assert_allclose(vals, [0.0] + [1.0] * 7 + [2.0], atol=1e-12)


def test_invariants(oracle_mod):
    g = G.chung_lu_typed(300, 8.0, 2.2, 60.0, 3, seed=4)
    rows = oracle_mod.all_edge_rows(g)
    w = oracle_mod.graphlet_edge_weights(g, rows, 1, (0, 1, 2))   # typed 3-paths {0,1,2}
    assert w.sum() > 0
    vals, vecs, nodes = oracle_mod.laplacian_spectrum(g, w)
    act = np.zeros(g.n, dtype=bool)
    act[nodes] = True
    assert vals[0] > -1e-12 and vals[-1] < 2 + 1e-12
    # scaling W does not change L
    vals3, _, _ = oracle_mod.laplacian_spectrum(g, w * np.uint64(3))
    np.testing.assert_allclose(vals, vals3, atol=1e-12)
    # a connected weighted graph: the smallest eigenvector follows sqrt(degree)
    ring = _graph(10, [(i, (i + 1) % 10) for i in range(10)] + [(0, 5)], [0] * 10, 1)
    wr = np.arange(1, ring.m + 1, dtype=np.uint64)
    v, U, a = oracle_mod.laplacian_spectrum(ring, wr)
    uv = ring.edges()
    deg = np.zeros(10)
    np.add.at(deg, uv[:, 0], wr.astype(float))
    np.add.at(deg, uv[:, 1], wr.astype(float))
    u0 = U[:, 0] * np.sign(U[0, 0])
    np.testing.assert_allclose(u0, np.sqrt(deg) / np.linalg.norm(np.sqrt(deg)), atol=1e-10)
    # embedding rows: unit length where the node is in an instance, else zero
    _, Z, comp = oracle_mod.embedding(g, w, 6)
    norms = np.sqrt((Z * Z).sum(axis=1))
    np.testing.assert_allclose(norms[act], 1.0, atol=1e-12)
    assert not norms[~act].any()
    np.testing.assert_array_equal(comp >= 0, act)


def test_per_component(oracle_mod):
    """Sec. 8.8: one embedding per component of G^H.  A triangle, a single
    edge, a 3-path and a 5-cycle (nodes shuffled), an isolated node, and a
    zero-weight edge joining the triangle to the cycle: each component has
    its own closed-form spectrum, a component of s <= D nodes gets all its s
    eigenvectors (so its rows of Z are orthonormal), and the zero-weight
    edge is in no component."""
    perm = np.random.default_rng(3).permutation(15)
    groups = {"tri": [0, 1, 2], "edge": [3, 4], "path": [5, 6, 7], "cyc": [8, 9, 10, 11, 12]}
    edges = [(0, 1), (1, 2), (0, 2), (3, 4), (5, 6), (6, 7),
             (8, 9), (9, 10), (10, 11), (11, 12), (8, 12), (2, 8)]
    pe = sorted(tuple(sorted((int(perm[a]), int(perm[b])))) for a, b in edges)
    g = _graph(15, pe, [0] * 15, 1)
    zero = tuple(sorted((int(perm[2]), int(perm[8]))))
    w = np.array([0 if tuple(e) == zero else 1 for e in g.edges().tolist()], dtype=np.uint64)
    ev, Z, comp = oracle_mod.embedding(g, w, 4)
    want = {"tri": [0, 1.5, 1.5], "edge": [0, 2], "path": [0, 1, 2],
            "cyc": list(np.sort(1 - np.cos(2 * np.pi * np.arange(5) / 5))[:4])}
    for name, ids in groups.items():
        nodes = perm[ids]
        r = int(nodes.min())
        assert set(comp[nodes].tolist()) == {r}
        k = len(want[name])
        np.testing.assert_allclose(ev[r, :k], want[name], atol=1e-12)
        assert not ev[r, k:].any()
        Zc = Z[nodes]
        if len(ids) <= 4:
            np.testing.assert_allclose(Zc @ Zc.T, np.eye(len(ids)), atol=1e-12)
            assert not Zc[:, len(ids):].any()
    for x in perm[[13, 14]]:
        assert comp[x] == -1 and not Z[x].any()
    # rows of ev that name no component are zero
    roots = {int(perm[ids].min()) for ids in groups.values()}
    assert not ev[[i for i in range(15) if i not in roots]].any()
