"""Oracle for directed typed graphlets (Sec. 4.8), test infrastructure only.

Sec. 4.8 extends the framework to directed graphs by splitting each typed
neighbourhood into typed out- and in-neighbourhoods, and with them the
sets T_ij^t, S_i^t, S_j^t of Alg. 1.  A pair of nodes joined both ways
(reciprocal arcs) is a third case here.  For every edge (i, j) of the
underlying undirected graph (canonical order, i < j) the oracle counts the
directed typed 3-node graphlets containing it:

  TRI[t][a][b]   nodes k of type t in T_ij with direction a between i and k
                 and direction b between j and k,
  PATH_I[t][a]   nodes k of type t in S_i (adjacent to i, not to j, k != j)
                 with direction a between i and k,
  PATH_J[t][b]   the same at j,

a, b in {0: out (the endpoint -> k), 1: in (k -> the endpoint), 2: both}.
Row layout: TRI at t*9 + a*3 + b, PATH_I at 9L + t*3 + a, PATH_J at
12L + t*3 + b (width 15L).

Global counts are per directed typed graphlet, i.e. per class of typed
digraphs under type-preserving isomorphism.  A class is named by its
canonical key: over every numbering of its nodes, the lexicographically
smallest tuple (types..., pair codes...), a pair code for nodes x < y
being 0 (no arc), 1 (x -> y), 2 (y -> x) or 3 (both).  Layout: the 2-node
classes at (t0*L + t1)*4 + c01, then the 3-node classes (3-paths and
triangles) at 4L^2 + ((t0*L + t1)*L + t2)*64 + c01*16 + c02*4 + c12;
entries that are not canonical keys stay zero.

Input: the underlying undirected graph (a tg_synth Graph) and `dirs`, one
byte per CSR slot (u -> col[s]): bit 0 the arc u -> col[s], bit 1 the arc
col[s] -> u.
"""

from __future__ import annotations

import itertools

import numpy as np


def row_width(L: int) -> int:
    return 15 * L


def global_width(L: int) -> int:
    return 4 * L * L + 64 * L ** 3


def _arcs(g, dirs):
    """Set of arcs (u, v) and the neighbour sets of the underlying graph."""
    arcs = set()
    nbr = [set() for _ in range(g.n)]
    for u in range(g.n):
        for s in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            x = int(g.col[s])
            nbr[u].add(x)
            if dirs[s] & 1:
                arcs.add((u, x))
            if dirs[s] & 2:
                arcs.add((x, u))
    return arcs, nbr


def _code(arcs, x, y):
    """Direction between endpoint x and node y: 0 out, 1 in, 2 both."""
    out, inn = (x, y) in arcs, (y, x) in arcs
    return 2 if out and inn else 0 if out else 1


def edge_rows(g, dirs) -> np.ndarray:
    """Per-edge directed typed 3-node counts (uint64 [M, 15L])."""
    L = g.L
    arcs, nbr = _arcs(g, dirs)
    uv = g.edges()
    rows = np.zeros((uv.shape[0], row_width(L)), dtype=np.uint64)
    ty = [int(t) for t in g.types]
    for e, (i, j) in enumerate(uv.tolist()):
        for k in nbr[i] & nbr[j]:
            rows[e, ty[k] * 9 + _code(arcs, i, k) * 3 + _code(arcs, j, k)] += 1
        for k in nbr[i] - nbr[j] - {j}:
            rows[e, 9 * L + ty[k] * 3 + _code(arcs, i, k)] += 1
        for k in nbr[j] - nbr[i] - {i}:
            rows[e, 12 * L + ty[k] * 3 + _code(arcs, j, k)] += 1
    return rows


def canonical(types, arcs_local):
    """Canonical key of a typed digraph on nodes 0..k-1 (k = 2 or 3):
    the smallest (types..., pair codes...) over all numberings."""
    k = len(types)
    best = None
    for perm in itertools.permutations(range(k)):      # new node q is old perm[q]
        t = tuple(int(types[perm[q]]) for q in range(k))
        codes = []
        for x, y in itertools.combinations(range(k), 2):
            c = (1 if (perm[x], perm[y]) in arcs_local else 0) + \
                (2 if (perm[y], perm[x]) in arcs_local else 0)
            codes.append(c)
        key = t + tuple(codes)
        if best is None or key < best:
            best = key
    return best


def key_index(key, L: int) -> int:
    if len(key) == 3:                     # (t0, t1, c01)
        t0, t1, c = key
        return (t0 * L + t1) * 4 + c
    t0, t1, t2, c01, c02, c12 = key
    return 4 * L * L + ((t0 * L + t1) * L + t2) * 64 + c01 * 16 + c02 * 4 + c12


def global_brute_force(g, dirs) -> np.ndarray:
    """Global counts by enumerating every edge and every connected 3-node
    subset (the definition; small graphs only)."""
    L = g.L
    arcs, nbr = _arcs(g, dirs)
    out = np.zeros(global_width(L), dtype=np.uint64)
    for (u, v) in g.edges().tolist():
        loc = {(0, 1)} if (u, v) in arcs else set()
        if (v, u) in arcs:
            loc.add((1, 0))
        out[key_index(canonical((g.types[u], g.types[v]), loc), L)] += 1
    for tri in itertools.combinations(range(g.n), 3):
        pairs = sum(1 for x, y in itertools.combinations(tri, 2) if y in nbr[x])
        if pairs < 2:
            continue
        loc = {(a, b) for a in range(3) for b in range(3) if a != b and (tri[a], tri[b]) in arcs}
        out[key_index(canonical([g.types[x] for x in tri], loc), L)] += 1
    return out


def _dir_arcs(end: int, code: int):
    """Arcs between endpoint `end` (node 0 or 1) and node 2 for a row's
    direction code (0 out, 1 in, 2 both)."""
    out, inn = (end, 2), (2, end)
    return {out} if code == 0 else {inn} if code == 1 else {out, inn}


def global_from_rows(g, dirs, rows) -> np.ndarray:
    """Global counts from the per-edge rows: each column of an edge names the
    class of its instances (nodes i = 0, j = 1, k = 2); a triangle is met
    from its 3 edges, a 3-path from its 2, so each 3-node class's sum is
    divided by its edge count."""
    L = g.L
    arcs, _ = _arcs(g, dirs)
    acc = np.zeros(global_width(L), dtype=object)
    for e, (i, j) in enumerate(g.edges().tolist()):
        eij = {(0, 1)} if (i, j) in arcs else set()
        if (j, i) in arcs:
            eij.add((1, 0))
        ti, tj = int(g.types[i]), int(g.types[j])
        acc[key_index(canonical((ti, tj), eij), L)] += 1
        for c in np.flatnonzero(rows[e]).tolist():
            if c < 9 * L:
                t, a, b = c // 9, (c // 3) % 3, c % 3
                loc = eij | _dir_arcs(0, a) | _dir_arcs(1, b)
            elif c < 12 * L:
                t, a = (c - 9 * L) // 3, (c - 9 * L) % 3
                loc = eij | _dir_arcs(0, a)
            else:
                t, b = (c - 12 * L) // 3, (c - 12 * L) % 3
                loc = eij | _dir_arcs(1, b)
            acc[key_index(canonical((ti, tj, t), loc), L)] += int(rows[e, c])
    out = np.zeros(global_width(L), dtype=np.uint64)
    for q in np.flatnonzero(acc).tolist():
        v = int(acc[q])
        if q >= 4 * L * L:
            codes = ((q - 4 * L * L) % 64) // 16, ((q - 4 * L * L) % 16) // 4, (q - 4 * L * L) % 4
            edges = sum(1 for c in codes if c)
            assert v % edges == 0, (q, v, edges)
            v //= edges
        out[q] = v
    return out


def edge_row(g, dirs, i: int, j: int) -> np.ndarray:
    """The row of one edge (i < j) straight from the CSR slices (for samples
    of large graphs)."""
    L = g.L
    rp, col = g.row_ptr, g.col
    ni, di = col[rp[i]:rp[i + 1]].astype(np.int64), dirs[rp[i]:rp[i + 1]]
    nj, dj = col[rp[j]:rp[j + 1]].astype(np.int64), dirs[rp[j]:rp[j + 1]]
    code = np.array([0, 0, 1, 2])          # direction bits 1, 2, 3 -> out, in, both
    row = np.zeros(row_width(L), dtype=np.uint64)
    common, pi, pj = np.intersect1d(ni, nj, assume_unique=True, return_indices=True)
    for k, a, b in zip(common.tolist(), code[di[pi]].tolist(), code[dj[pj]].tolist()):
        row[int(g.types[k]) * 9 + a * 3 + b] += 1
    only_i = ~np.isin(ni, nj) & (ni != j)
    for k, a in zip(ni[only_i].tolist(), code[di[only_i]].tolist()):
        row[9 * L + int(g.types[k]) * 3 + a] += 1
    only_j = ~np.isin(nj, ni) & (nj != i)
    for k, b in zip(nj[only_j].tolist(), code[dj[only_j]].tolist()):
        row[12 * L + int(g.types[k]) * 3 + b] += 1
    return row
