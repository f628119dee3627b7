"""Exhaustive typed-graphlet counter for tiny graphs (a pin for the oracle).

It shares nothing with the oracle: every 3- and 4-node subset of V is
tested, connected induced 4-node subgraphs are matched against explicit
graphlet templates by trying all 24 node bijections, and the edge's orbit is
read off the template.  Templates are the six connected 4-node graphs of the
paper's Table 3 with their edge orbits:

  4-path 0-1-2-3 ........ end edges g3, centre edge g4
  4-star centre 0 ....... g5
  4-cycle 0-1-2-3-0 ..... g6
  tailed triangle 0,1,2 + tail 2-3:  tail (2,3) g7; (0,1), the triangle
                          edge away from the tail's node, g8; (0,2),(1,2) g9
  diamond 0-1-2-3-0 + chord 0-2:  chord g11, the rest g10
  4-clique .............. g12

Global counts are counted directly as instances (each subset once), not
through per-edge sums.
"""

from __future__ import annotations

import itertools

import numpy as np

TEMPLATES = {
    # graphlet id h -> {edge(frozenset) -> orbit}
    3: {(0, 1): 3, (1, 2): 4, (2, 3): 3},
    4: {(0, 1): 5, (0, 2): 5, (0, 3): 5},
    5: {(0, 1): 6, (1, 2): 6, (2, 3): 6, (0, 3): 6},
    6: {(0, 1): 8, (0, 2): 9, (1, 2): 9, (2, 3): 7},
    7: {(0, 1): 10, (1, 2): 10, (2, 3): 10, (0, 3): 10, (0, 2): 11},
    8: {(0, 1): 12, (0, 2): 12, (0, 3): 12, (1, 2): 12, (1, 3): 12, (2, 3): 12},
}
_TEMPLATE_SETS = {h: {frozenset(e): o for e, o in es.items()} for h, es in TEMPLATES.items()}


def _match(nodes, adj):
    """(graphlet id, {frozenset(edge of G) -> orbit}) for a connected 4-set."""
    edges = [frozenset((a, b)) for a, b in itertools.combinations(nodes, 2) if adj[a][b]]
    es = set(edges)
    for h, tmpl in _TEMPLATE_SETS.items():
        if len(tmpl) != len(es):
            continue
        for perm in itertools.permutations(range(4)):
            mp = {nodes[p]: q for p, q in zip(range(4), perm)}
            img = {frozenset(mp[x] for x in e) for e in es}
            if img == set(tmpl):
                return h, {e: tmpl[frozenset(mp[x] for x in e)] for e in es}
    return None, None


def _connected(nodes, adj):
    seen = {nodes[0]}
    stack = [nodes[0]]
    while stack:
        a = stack.pop()
        for b in nodes:
            if b not in seen and adj[a][b]:
                seen.add(b)
                stack.append(b)
    return len(seen) == len(nodes)


def _pairs(L):
    return [(t, u) for t in range(L) for u in range(t, L)]


def column_index(L):
    """name -> column, following the documented row layout."""
    names = {}
    for t in range(L):
        names[f"tri[{t}]"] = t
        names[f"path3[{t}]"] = L + t
    P = L * (L + 1) // 2
    for g in range(3, 13):
        for p, (t, u) in enumerate(_pairs(L)):
            names[f"g{g}[{t},{u}]"] = 2 * L + (g - 3) * P + p
    return names


def multisets(L, k):
    """Sorted type multisets of size k in co-lexicographic order."""
    ms = list(itertools.combinations_with_replacement(range(L), k))
    return sorted(ms, key=lambda m: tuple(reversed(m)))


def adjacency(n, edges):
    adj = [[False] * n for _ in range(n)]
    for a, b in edges:
        adj[a][b] = adj[b][a] = True
    return adj


def per_edge_rows(n, edges, types, L):
    """Rows for edges (canonical u < v, in the order given)."""
    adj = adjacency(n, edges)
    col = column_index(L)
    W = 2 * L + 10 * (L * (L + 1) // 2)
    rows = np.zeros((len(edges), W), dtype=np.uint64)
    index = {frozenset(e): q for q, e in enumerate(edges)}
    for q, (i, j) in enumerate(edges):
        for k in range(n):
            if k in (i, j):
                continue
            a, b = adj[i][k], adj[j][k]
            if a and b:
                rows[q, col[f"tri[{types[k]}]"]] += 1
            elif a or b:
                rows[q, col[f"path3[{types[k]}]"]] += 1
    for quad in itertools.combinations(range(n), 4):
        if not _connected(list(quad), adj):
            continue
        h, orbits = _match(list(quad), adj)
        assert h is not None
        for e, orb in orbits.items():
            q = index[e]
            k, r = [x for x in quad if x not in e]
            t, u = sorted((int(types[k]), int(types[r])))
            rows[q, col[f"g{orb}[{t},{u}]"]] += 1
    return rows


def global_instances(n, edges, types, L):
    """Instance counts of every typed 2-, 3- and 4-node graphlet.

    Layout: h0 | h1 (3-path) | h2 (triangle) | h3..h8, multisets in
    co-lexicographic order inside each block.
    """
    adj = adjacency(n, edges)
    r2 = {m: q for q, m in enumerate(multisets(L, 2))}
    r3 = {m: q for q, m in enumerate(multisets(L, 3))}
    r4 = {m: q for q, m in enumerate(multisets(L, 4))}
    n2, n3, n4 = len(r2), len(r3), len(r4)
    out = np.zeros(n2 + 2 * n3 + 6 * n4, dtype=np.uint64)
    for a, b in edges:
        out[r2[tuple(sorted((int(types[a]), int(types[b]))))]] += 1
    for tri in itertools.combinations(range(n), 3):
        m = sum(adj[x][y] for x, y in itertools.combinations(tri, 2))
        key = r3[tuple(sorted(int(types[x]) for x in tri))]
        if m == 2:
            out[n2 + key] += 1
        elif m == 3:
            out[n2 + n3 + key] += 1
    for quad in itertools.combinations(range(n), 4):
        if not _connected(list(quad), adj):
            continue
        h, _ = _match(list(quad), adj)
        key = r4[tuple(sorted(int(types[x]) for x in quad))]
        out[n2 + 2 * n3 + (h - 3) * n4 + key] += 1
    return out
