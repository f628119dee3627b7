"""Pins of the directed typed graphlet oracle (Sec. 4.8).

* Collapsing the direction splits gives the undirected typed counts of the
  pinned undirected oracle: sum over (a, b) of TRI[t][a][b] = tri[t] and
  PATH_I + PATH_J summed over directions = path3[t].
* Per-edge rows against a brute force that scans every node k with an
  adjacency matrix (no neighbour sets).
* Global counts from the rows against an enumeration of every edge and
  every connected 3-node subset.
* The canonical keys reproduce the classical triad census: 16 classes of
  3-node digraphs, 13 of them connected; 2 of 2-node ones (L = 1).
* Hand-worked examples: a directed 3-cycle, a transitive triangle, and a
  3-path through a reciprocal pair, worked out from the row and key
  definitions.
"""

import itertools

import numpy as np
import pytest

from tg_synth import graphs as G


@pytest.fixture(scope="module")
def D(oracle_mod):
    return oracle_mod.directed


def _hand(n, arcs, types, L):
    """A digraph from an arc list: underlying CSR and per-slot direction bits."""
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


def test_collapse_to_undirected(oracle_mod, D):
    rng = np.random.default_rng(5)
    for s in range(30):
        n = int(rng.integers(4, 12))
        L = int(rng.integers(1, 4))
        g = G.random_small_graph(n, float(rng.uniform(0.2, 0.9)), L, 300 + s)
        if g.m == 0:
            continue
        dirs = G.orient(g, float(rng.uniform(0, 1)), s)
        rows = D.edge_rows(g, dirs).astype(np.int64)
        und = oracle_mod.all_edge_rows(g).astype(np.int64)
        names = oracle_mod.column_names(L)
        for t in range(L):
            tri = rows[:, t * 9:(t + 1) * 9].sum(axis=1)
            path = rows[:, 9 * L + 3 * t:9 * L + 3 * t + 3].sum(axis=1) + \
                rows[:, 12 * L + 3 * t:12 * L + 3 * t + 3].sum(axis=1)
            np.testing.assert_array_equal(tri, und[:, names.index(f"tri[{t}]")])
            np.testing.assert_array_equal(path, und[:, names.index(f"path3[{t}]")])


def test_rows_brute_force(D):
    rng = np.random.default_rng(6)
    for s in range(25):
        n = int(rng.integers(3, 10))
        L = int(rng.integers(1, 4))
        g = G.random_small_graph(n, float(rng.uniform(0.3, 1.0)), L, 500 + s)
        if g.m == 0:
            continue
        dirs = G.orient(g, float(rng.uniform(0, 1)), 77 + s)
        A = np.zeros((n, n), dtype=np.int64)        # A[u][v] = 1 iff arc u -> v
        for u in range(n):
            for q in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
                v = int(g.col[q])
                A[u, v] |= int(dirs[q] & 1)
                A[v, u] |= int(dirs[q] >> 1 & 1)
        U = (A + A.T) > 0
        want = np.zeros((g.m, 15 * L), dtype=np.uint64)
        for e, (i, j) in enumerate(g.edges().tolist()):
            for k in range(n):
                if k in (i, j):
                    continue
                ci = 2 if A[i, k] and A[k, i] else 0 if A[i, k] else 1
                cj = 2 if A[j, k] and A[k, j] else 0 if A[j, k] else 1
                t = int(g.types[k])
                if U[i, k] and U[j, k]:
                    want[e, t * 9 + ci * 3 + cj] += 1
                elif U[i, k]:
                    want[e, 9 * L + t * 3 + ci] += 1
                elif U[j, k]:
                    want[e, 12 * L + t * 3 + cj] += 1
        np.testing.assert_array_equal(D.edge_rows(g, dirs), want)


def test_global_two_ways(D):
    rng = np.random.default_rng(7)
    for s in range(25):
        n = int(rng.integers(3, 11))
        L = int(rng.integers(1, 4))
        g = G.random_small_graph(n, float(rng.uniform(0.2, 0.9)), L, 700 + s)
        dirs = G.orient(g, float(rng.uniform(0, 1)), s)
        rows = D.edge_rows(g, dirs)
        np.testing.assert_array_equal(D.global_from_rows(g, dirs, rows),
                                      D.global_brute_force(g, dirs))


def test_triad_census(D):
    pairs = [(0, 1), (1, 0), (0, 2), (2, 0), (1, 2), (2, 1)]
    every, connected = set(), set()
    for bits in range(64):
        loc = {pairs[q] for q in range(6) if bits >> q & 1}
        key = D.canonical((0, 0, 0), loc)
        every.add(key)
        if len({tuple(sorted(a)) for a in loc}) >= 2:
            connected.add(key)
    assert len(every) == 16 and len(connected) == 13
    two = {D.canonical((0, 0), loc) for loc in ({(0, 1)}, {(1, 0)}, {(0, 1), (1, 0)})}
    assert len(two) == 2
    # with two types a single arc between different types has two classes
    two = {D.canonical((0, 1), loc) for loc in ({(0, 1)}, {(1, 0)}, {(0, 1), (1, 0)})}
    assert len(two) == 3


def test_hand_examples(D):
    # directed 3-cycle 0 -> 1 -> 2 -> 0, one type
    g, dirs = _hand(3, [(0, 1), (1, 2), (2, 0)], [0, 0, 0], 1)
    rows = D.edge_rows(g, dirs)
    want = np.zeros((3, 15), dtype=np.uint64)
    want[0, 1 * 3 + 0] = 1      # edge (0,1), k = 2: in at 0 (2 -> 0), out at 1 (1 -> 2)
    want[1, 0 * 3 + 1] = 1      # edge (0,2), k = 1: out at 0, in at 2 (1 -> 2)
    want[2, 1 * 3 + 0] = 1      # edge (1,2), k = 0: in at 1 (0 -> 1), out at 2 (2 -> 0)
    np.testing.assert_array_equal(rows, want)
    glob = D.global_brute_force(g, dirs)
    assert glob[1] == 3                            # 3 arcs, key (0, 0, 1)
    assert glob[4 + 1 * 16 + 2 * 4 + 1] == 1      # cyclic triangle, key (0,0,0, 1,2,1)
    assert glob.sum() == 4
    # transitive triangle 0 -> 1, 0 -> 2, 1 -> 2
    g, dirs = _hand(3, [(0, 1), (0, 2), (1, 2)], [0, 0, 0], 1)
    rows = D.edge_rows(g, dirs)
    assert rows[0, 0] == 1 and rows[1, 1] == 1 and rows[2, 4] == 1 and rows.sum() == 3
    glob = D.global_brute_force(g, dirs)
    assert glob[4 + 16 + 4 + 1] == 1 and glob[1] == 3 and glob.sum() == 4
    # 3-path 0 <-> 1 -> 2, types (0, 1, 0), L = 2
    g, dirs = _hand(3, [(0, 1), (1, 0), (1, 2)], [0, 1, 0], 2)
    rows = D.edge_rows(g, dirs)
    want = np.zeros((2, 30), dtype=np.uint64)
    want[0, 24 + 0] = 1         # edge (0,1): k = 2 in S_j, type 0, out at 1
    want[1, 18 + 2] = 1         # edge (1,2): k = 0 in S_i, type 0, both at 1
    np.testing.assert_array_equal(rows, want)
    glob = D.global_brute_force(g, dirs)
    assert glob[(0 * 2 + 1) * 4 + 3] == 1         # reciprocal pair, types (0, 1)
    assert glob[(0 * 2 + 1) * 4 + 2] == 1         # arc 1 -> 2: key (0, 1, 2)
    assert glob[16 + 1 * 64 + 2 * 4 + 3] == 1     # the 3-path, key (0,0,1, 0,2,3)
    assert glob.sum() == 3


def test_single_edge_rows(D):
    """The CSR-slice form of one edge's row equals the set-based rows."""
    g = G.chung_lu_typed(300, 8.0, 2.2, 40.0, 3, seed=9)
    dirs = G.orient(g, 0.25, 4)
    rows = D.edge_rows(g, dirs)
    for e, (i, j) in enumerate(g.edges().tolist()):
        np.testing.assert_array_equal(D.edge_row(g, dirs, i, j), rows[e])
