"""Oracle for typed-graphlet spectral node embeddings (Alg. 5), test
infrastructure only.

Alg. 5 for one typed graphlet H:
  1. W_ij = number of instances of H that contain the edge (i, j), for every
     edge (i, j) of G;
  2. D_ii = sum_j W_ij, the typed-graphlet degree;
  3. the eigenvectors u_1..u_D of the D smallest eigenvalues of the
     normalised Laplacian L = I - D^{-1/2} W D^{-1/2};
  4. Z_ij = U_ij / sqrt(sum_j U_ij^2), each row scaled to unit length.
Sec. 8.8 runs the algorithm on each connected component of the typed
graphlet graph G^H (the edges with W_ij > 0) and stores each component's
embedding in its nodes' rows of Z; a component of s < D nodes has s
eigenvectors, and its rows are zero past column s.

Readings (listed in the design notes): nodes with D_ii = 0 belong to no
instance of H and to no component; their rows are zero.  A component is
named by its smallest node id.

W comes from the oracle's typed per-edge rows: the orbits of H's graphlet
(Sec. 4.4's orbit-to-graphlet map, written out here) summed over the type
pairs that complete the edge's endpoint types to H's type multiset.  The
components come from a breadth-first search; each eigenproblem is dense,
in float64, by numpy.linalg.eigh.
"""

from __future__ import annotations

from collections import deque

import numpy as np

from .oracle import column_names

# orbits of each graphlet id (h0 edge, h1 3-path, h2 triangle, h3..h8 4-node)
ORBITS = {1: ["path3"], 2: ["tri"], 3: ["g3", "g4"], 4: ["g5"], 5: ["g6"],
          6: ["g7", "g8", "g9"], 7: ["g10", "g11"], 8: ["g12"]}


def graphlet_edge_weights(g, rows: np.ndarray, graphlet: int, types_sorted) -> np.ndarray:
    """W_e for every edge (rows of all edges in canonical order): instances
    of the typed graphlet (graphlet, sorted type multiset) containing e."""
    L = g.L
    uv = g.edges()
    want = tuple(sorted(int(t) for t in types_sorted))
    a = g.types[uv[:, 0]].astype(np.int64)
    b = g.types[uv[:, 1]].astype(np.int64)
    w = np.zeros(uv.shape[0], dtype=np.uint64)
    if graphlet == 0:
        for e in range(uv.shape[0]):
            w[e] = 1 if tuple(sorted((a[e], b[e]))) == want else 0
        return w
    names = column_names(L)
    idx = {n: q for q, n in enumerate(names)}
    for e in range(uv.shape[0]):
        total = 0
        for orb in ORBITS[graphlet]:
            if graphlet <= 2:
                for t in range(L):
                    if tuple(sorted((a[e], b[e], t))) == want:
                        total += int(rows[e, idx[f"{orb}[{t}]"]])
            else:
                for t in range(L):
                    for u in range(t, L):
                        if tuple(sorted((a[e], b[e], t, u))) == want:
                            total += int(rows[e, idx[f"{orb}[{t},{u}]"]])
        w[e] = total
    return w


def _sub_adjacency(g, weights: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """Dense weighted adjacency among `nodes` (in that order)."""
    uv = g.edges()
    pos = np.full(g.n, -1, dtype=np.int64)
    pos[nodes] = np.arange(nodes.shape[0])
    a, b = pos[uv[:, 0]], pos[uv[:, 1]]
    keep = (a >= 0) & (b >= 0)
    Wa = np.zeros((nodes.shape[0], nodes.shape[0]))
    w = weights.astype(np.float64)[keep]
    Wa[a[keep], b[keep]] = w
    Wa[b[keep], a[keep]] = w
    return Wa


def components(g, weights: np.ndarray) -> np.ndarray:
    """Component of every node in G^H (the edges of nonzero weight), named
    by its smallest node id; -1 for nodes on no such edge."""
    uv = g.edges()
    keep = weights > 0
    adj = [[] for _ in range(g.n)]
    for (u, v) in uv[keep].tolist():
        adj[u].append(v)
        adj[v].append(u)
    comp = np.full(g.n, -1, dtype=np.int64)
    for s in range(g.n):          # ascending: s is its component's smallest id
        if comp[s] >= 0 or not adj[s]:
            continue
        comp[s] = s
        q = deque([s])
        while q:
            u = q.popleft()
            for v in adj[u]:
                if comp[v] < 0:
                    comp[v] = s
                    q.append(v)
    return comp


def laplacian_spectrum(g, weights: np.ndarray, nodes=None):
    """(eigenvalues ascending, eigenvectors as columns, node ids) of the
    normalised Laplacian of the weighted graph on `nodes` (default: every
    node of nonzero weighted degree)."""
    if nodes is None:
        uv = g.edges()
        deg = np.zeros(g.n)
        np.add.at(deg, uv[:, 0], weights.astype(np.float64))
        np.add.at(deg, uv[:, 1], weights.astype(np.float64))
        nodes = np.flatnonzero(deg > 0)
    nodes = np.asarray(nodes, dtype=np.int64)
    Wa = _sub_adjacency(g, weights, nodes)
    da = Wa.sum(axis=1)
    s = 1.0 / np.sqrt(da)
    Lap = np.eye(nodes.shape[0]) - (s[:, None] * Wa) * s[None, :]
    vals, vecs = np.linalg.eigh(Lap)
    return vals, vecs, nodes


def embedding(g, weights: np.ndarray, dim: int, raw: bool = False):
    """Alg. 5 per component of G^H: (eigenvalues float64 [n, dim] with
    component r's spectrum in row r, Z [n, dim], component [n]).  With
    `raw`, Z holds the eigenvectors U before the row scaling."""
    comp = components(g, weights)
    U = np.zeros((g.n, dim))
    ev = np.zeros((g.n, dim))
    for r in np.unique(comp[comp >= 0]):
        nodes = np.flatnonzero(comp == r)
        vals, vecs, _ = laplacian_spectrum(g, weights, nodes)
        k = min(dim, nodes.shape[0])
        U[nodes, :k] = vecs[:, :k]
        ev[r, :k] = vals[:k]
    if raw:
        return ev, U, comp
    norm = np.sqrt((U * U).sum(axis=1))
    Z = np.divide(U, norm[:, None], out=np.zeros_like(U), where=norm[:, None] > 0)
    return ev, Z, comp
