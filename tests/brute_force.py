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


# ------------------------------------------------ position-aware (Sec. 5)
#
# Templates with numbered positions (the same drawings as above):
#   3: 4-path 0-1-2-3; 4: 4-star centre 0; 5: 4-cycle 0-1-2-3-0;
#   6: tailed triangle 0,1,2 with tail 2-3; 7: chordal cycle 0-1-2-3-0
#   with chord 0-2; 8: 4-clique.
# For an edge of a matched template, seen oriented (i at template position
# pi, j at pj), ROLE gives the block of the position-aware row and the
# positions whose types are its (x, y) key (ordered), or the two positions
# of an unordered key.  It is written from the drawings, position by
# position, not from the sets S_i, S_j, T and I.

PA_PAIR = {"g5i", "g5j", "g7i", "g7j", "g11", "g12"}


def _cyc_next(p, other):
    """Cycle 0-1-2-3-0: the neighbour of p that is not `other`."""
    a, b = (p + 1) % 4, (p + 3) % 4
    return a if b == other else b


def role(h, pi, pj):
    if h == 3:                                   # path 0-1-2-3
        e = {pi, pj}
        if e == {1, 2}:                          # centre edge: x hangs at i, y at j
            return "g4", pi - 1 if pi == 1 else 3, pj - 1 if pj == 1 else 3
        if e == {0, 1}:                          # the path continues from position 1
            return ("g3i" if pi == 1 else "g3j"), 2, 3
        return ("g3i" if pi == 2 else "g3j"), 1, 0  # edge {2, 3}, continues from 2
    if h == 4:                                   # star, centre 0
        others = [q for q in (1, 2, 3) if q not in (pi, pj)]
        return ("g5i" if pi == 0 else "g5j"), others[0], others[1]
    if h == 5:                                   # cycle
        return "g6", _cyc_next(pi, pj), _cyc_next(pj, pi)
    if h == 6:                                   # triangle 0,1,2; tail 2-3
        e = {pi, pj}
        if e == {2, 3}:                          # the tail edge
            return ("g7i" if pi == 2 else "g7j"), 0, 1
        if e == {0, 1}:                          # triangle edge away from the tail
            return "g8", 2, 3
        third = ({0, 1} - e).pop()               # triangle edge at position 2
        return ("g9i" if pi == 2 else "g9j"), third, 3
    if h == 7:                                   # cycle 0-1-2-3-0, chord 0-2
        e = {pi, pj}
        if e == {0, 2}:
            return "g11", 1, 3
        chord_end = pi if pi in (0, 2) else pj   # the outer edge's chord end
        rim = pj if chord_end == pi else pi
        return ("g10i" if chord_end == pi else "g10j"), 2 - chord_end, 4 - rim
    others = [q for q in range(4) if q not in (pi, pj)]
    return "g12", others[0], others[1]


def pa_column_index(L):
    """name -> column of the documented position-aware row layout."""
    names, c = {}, 0
    for b in ["tri", "path_i", "path_j"]:
        for t in range(L):
            names[f"{b}[{t}]"] = c
            c += 1
    for b in ["g3i", "g3j", "g4", "g5i", "g5j", "g6", "g7i", "g7j", "g8", "g9i", "g9j", "g10i",
              "g10j", "g11", "g12"]:
        if b in PA_PAIR:
            for t, u in _pairs(L):
                names[f"{b}{{{t},{u}}}"] = c
                c += 1
        else:
            for x in range(L):
                for y in range(L):
                    names[f"{b}[{x},{y}]"] = c
                    c += 1
    return names


def _matches(nodes, adj):
    """All bijections (node -> template position) onto the matching template."""
    edges = {frozenset((a, b)) for a, b in itertools.combinations(nodes, 2) if adj[a][b]}
    for h, tmpl in _TEMPLATE_SETS.items():
        if len(tmpl) != len(edges):
            continue
        out = []
        for perm in itertools.permutations(range(4)):
            mp = {nodes[p]: q for p, q in zip(range(4), perm)}
            if {frozenset(mp[x] for x in e) for e in edges} == set(tmpl):
                out.append(mp)
        if out:
            return h, out
    return None, []


def pa_per_edge_rows(n, edges, types, L):
    """Position-aware rows for edges in the orientation given (i, j)."""
    adj = adjacency(n, edges)
    col = pa_column_index(L)
    rows = np.zeros((len(edges), len(col)), dtype=np.uint64)
    for q, (i, j) in enumerate(edges):
        for k in range(n):
            if k in (i, j):
                continue
            a, b = adj[i][k], adj[j][k]
            t = int(types[k])
            if a and b:
                rows[q, col[f"tri[{t}]"]] += 1
            elif a:
                rows[q, col[f"path_i[{t}]"]] += 1
            elif b:
                rows[q, col[f"path_j[{t}]"]] += 1
    where = {}
    for q, (i, j) in enumerate(edges):
        where[frozenset((i, j))] = q
    for quad in itertools.combinations(range(n), 4):
        if not _connected(list(quad), adj):
            continue
        h, maps = _matches(list(quad), adj)
        mp = maps[0]
        pos_node = {p: v for v, p in mp.items()}
        for e, q in where.items():
            if not e <= set(quad):
                continue
            i, j = edges[q]
            block, px, py = role(h, mp[i], mp[j])
            tx, ty = int(types[pos_node[px]]), int(types[pos_node[py]])
            if block in PA_PAIR:
                tx, ty = sorted((tx, ty))
                rows[q, col[f"{block}{{{tx},{ty}}}"]] += 1
            else:
                rows[q, col[f"{block}[{tx},{ty}]"]] += 1
    return rows


def _canon(h, maps, types):
    """Smallest types-by-position tuple over every matching bijection (the
    class of the typed instance under type-preserving isomorphism)."""
    best = None
    for mp in maps:
        lab = [0] * 4
        for v, p in mp.items():
            lab[p] = int(types[v])
        lab = tuple(lab)
        if best is None or lab < best:
            best = lab
    return best


def pa_global_instances(n, edges, types, L):
    """Instance counts per class, keyed (graphlet, canonical labelling):
    h0 (sorted pair), h1 (centre, sorted ends), h2 (sorted triple), h3..h8
    the smallest types-by-position tuple over the template's matches."""
    adj = adjacency(n, edges)
    out = {}

    def add(key):
        out[key] = out.get(key, 0) + 1

    for a, b in edges:
        add((0, tuple(sorted((int(types[a]), int(types[b]))))))
    for tri in itertools.combinations(range(n), 3):
        es = [(x, y) for x, y in itertools.combinations(tri, 2) if adj[x][y]]
        if len(es) == 3:
            add((2, tuple(sorted(int(types[x]) for x in tri))))
        elif len(es) == 2:
            centre = [x for x in tri if all(x in e for e in es)][0]
            ends = sorted(int(types[x]) for x in tri if x != centre)
            add((1, (int(types[centre]), ends[0], ends[1])))
    for quad in itertools.combinations(range(n), 4):
        if not _connected(list(quad), adj):
            continue
        h, maps = _matches(list(quad), adj)
        add((h, _canon(h, maps, types)))
    return out


def pa_class_key(h, lab, L):
    """The brute force's class key of a types-by-position labelling of
    graphlet h (as pa_global_instances keys it)."""
    if h == 0:
        return (0, tuple(sorted(lab)))
    if h == 2:
        return (2, tuple(sorted(lab)))
    if h == 1:
        return (1, (lab[0],) + tuple(sorted(lab[1:])))
    # every position permutation that maps the template onto itself
    tmpl = set(_TEMPLATE_SETS[h])
    best = None
    for perm in itertools.permutations(range(4)):
        if {frozenset(perm[x] for x in e) for e in tmpl} != tmpl:
            continue
        img = [0] * 4
        for q in range(4):
            img[perm[q]] = lab[q]
        img = tuple(img)
        if best is None or img < best:
            best = img
    return (h, best)
