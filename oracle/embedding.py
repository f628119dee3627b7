"""Oracle for typed-graphlet spectral node embeddings (Alg. 5), test
infrastructure only.

Alg. 5 for one typed graphlet H:
  1. W_ij = number of instances of H that contain the edge (i, j), for every
     edge (i, j) of G;
  2. D_ii = sum_j W_ij, the typed-graphlet degree;
  3. the eigenvectors u_1..u_D of the D smallest eigenvalues of the
     normalised Laplacian L = I - D^{-1/2} W D^{-1/2};
  4. Z_ij = U_ij / sqrt(sum_j U_ij^2), each row scaled to unit length.

Readings (listed in the design notes): nodes with D_ii = 0 belong to no
instance of H and keep a zero row; the Laplacian is that of the whole
weighted graph on the other nodes (a graph with several components has one
zero eigenvalue per component).

W comes from the oracle's typed per-edge rows: the orbits of H's graphlet
(Sec. 4.4's orbit-to-graphlet map, written out here) summed over the type
pairs that complete the edge's endpoint types to H's type multiset.  The
eigenproblem is dense, in float64, by numpy.linalg.eigh.
"""

from __future__ import annotations

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


def laplacian_spectrum(g, weights: np.ndarray):
    """(eigenvalues ascending, eigenvectors as columns, active mask) of the
    normalised Laplacian of the weighted graph on the nodes of nonzero
    weighted degree."""
    uv = g.edges()
    n = g.n
    Wd = np.zeros((n, n))
    w = weights.astype(np.float64)
    Wd[uv[:, 0], uv[:, 1]] = w
    Wd[uv[:, 1], uv[:, 0]] = w
    deg = Wd.sum(axis=1)
    act = deg > 0
    Wa = Wd[np.ix_(act, act)]
    s = 1.0 / np.sqrt(deg[act])
    Lap = np.eye(int(act.sum())) - (s[:, None] * Wa) * s[None, :]
    vals, vecs = np.linalg.eigh(Lap)
    return vals, vecs, act


def embedding(g, weights: np.ndarray, dim: int):
    """(the dim smallest Laplacian eigenvalues, Z [n, dim]) of Alg. 5."""
    vals, vecs, act = laplacian_spectrum(g, weights)
    k = min(dim, vals.shape[0])
    U = np.zeros((g.n, dim))
    U[act, :k] = vecs[:, :k]
    norm = np.sqrt((U * U).sum(axis=1))
    Z = np.divide(U, norm[:, None], out=np.zeros_like(U), where=norm[:, None] > 0)
    return vals[:k], Z
