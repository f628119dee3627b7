"""Pins of the CPU oracle against things other than itself.

* brute force over every 4-node subset with graphlet templates (tiny graphs);
* hand-worked fixtures (tests/golden/hand_graphs.json);
* closed forms on complete, complete bipartite, cycle, star and Petersen
  graphs;
* invariants: Prop. 1 (typed counts sum to the untyped count), the corrected
  Property prop:1 (d_i + d_j = 2|T| + |S_i| + |S_j| + 2), Lemma sums,
  relabelling invariance, type-permutation equivariance, and the global
  division by |E(H)| of Problem 2.
"""

import itertools
import json
import os

import numpy as np
import pytest

import brute_force as BF
from tg_synth import graphs as G

HERE = os.path.dirname(os.path.abspath(__file__))


def graph_from_edges(n, edges, types, L):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    rp, col = G.csr_from_edges(n, e[:, 0], e[:, 1])
    return G.Graph(rp, col, np.asarray(types, dtype=np.uint8), L, "hand")


def named(L, names_to_values):
    idx = BF.column_index(L)
    W = 2 * L + 10 * (L * (L + 1) // 2)
    row = np.zeros(W, dtype=np.uint64)
    for k, v in names_to_values.items():
        row[idx[k]] = v
    return row


def global_named(L, d):
    r2 = {m: q for q, m in enumerate(BF.multisets(L, 2))}
    r3 = {m: q for q, m in enumerate(BF.multisets(L, 3))}
    r4 = {m: q for q, m in enumerate(BF.multisets(L, 4))}
    n2, n3, n4 = len(r2), len(r3), len(r4)
    out = np.zeros(n2 + 2 * n3 + 6 * n4, dtype=np.uint64)
    for k, v in d.items():
        h = int(k[1])
        ts = tuple(int(x) for x in k[k.index("[") + 1:-1].split(","))
        if h == 0:
            out[r2[ts]] = v
        elif h in (1, 2):
            out[n2 + (h - 1) * n3 + r3[ts]] = v
        else:
            out[n2 + 2 * n3 + (h - 3) * n4 + r4[ts]] = v
    return out


# ------------------------------------------------------------ layout pins

def test_layout_widths(oracle_mod):
    for L in range(1, 10):
        P = L * (L + 1) // 2
        assert oracle_mod.row_width(L) == 2 * L + 10 * P
        assert oracle_mod.global_width(L) == len(BF.multisets(L, 2)) + 2 * len(
            BF.multisets(L, 3)) + 6 * len(BF.multisets(L, 4))
    # Table 2: C(L+K-1, K) typed graphlets of one K-node graphlet
    table2 = {2: [1, 3, 6, 10, 15, 21, 28, 36, 45],
              3: [1, 4, 10, 20, 35, 56, 84, 120, 165],
              4: [1, 5, 15, 35, 70, 126, 210, 330, 495]}
    for K, vals in table2.items():
        assert [len(BF.multisets(L, K)) for L in range(1, 10)] == vals
    # cora caption (L=7): 1428 possible typed 3- and 4-node graphlets
    assert oracle_mod.global_width(7) - len(BF.multisets(7, 2)) == 1428
    # space example (M=1e7, L=7, 4 bytes): 90.72 GB for all typed orbits
    n_orbit_keys = 2 * len(BF.multisets(7, 3)) + 10 * len(BF.multisets(7, 4))
    assert n_orbit_keys * 4 * 10**7 == 90_720_000_000


def test_pair_index(oracle_mod):
    for L in (1, 3, 5, 8):
        seen = []
        for t in range(L):
            for u in range(t, L):
                seen.append(oracle_mod.pair_index(L, t, u))
                assert oracle_mod.pair_index(L, u, t) == oracle_mod.pair_index(L, t, u)
        assert seen == list(range(L * (L + 1) // 2))


# ------------------------------------------------------- hand fixtures

def _hand_cases():
    with open(os.path.join(HERE, "golden", "hand_graphs.json")) as f:
        return json.load(f)["graphs"]


@pytest.mark.parametrize("case", _hand_cases(), ids=lambda c: c["name"].split(" ")[0])
@pytest.mark.parametrize("method", ["paper", "definition"])
def test_hand_graphs(oracle_mod, case, method):
    g = graph_from_edges(case["n"], case["edges"], case["types"], case["L"])
    L = case["L"]
    uv = g.edges()
    rows = oracle_mod.edge_rows(g, uv, method=method, threads=2)
    for q, (i, j) in enumerate(uv):
        want = named(L, case["rows"][f"{i},{j}"])
        np.testing.assert_array_equal(rows[q], want, err_msg=f"edge {i},{j}")
    glob = oracle_mod.global_counts(g, rows)
    np.testing.assert_array_equal(glob, global_named(L, case["global"]))


# ------------------------------------------------------ brute force pins

def _random_cases():
    cases = []
    seed = 0
    for n in (5, 7, 9, 10):
        for p in (0.25, 0.5, 0.8, 1.0):
            for L in (1, 2, 3, 4):
                cases.append((n, p, L, seed))
                seed += 1
    return cases


@pytest.mark.parametrize("n,p,L,seed", _random_cases())
def test_against_brute_force(oracle_mod, n, p, L, seed):
    g = G.random_small_graph(n, p, L, seed)
    uv = g.edges()
    if uv.shape[0] == 0:
        return
    want = BF.per_edge_rows(n, [tuple(e) for e in uv.tolist()], g.types, L)
    for method in ("paper", "definition"):
        got = oracle_mod.edge_rows(g, uv, method=method, threads=3)
        np.testing.assert_array_equal(got, want, err_msg=method)
        # the reverse orientation gives the same row
        back = oracle_mod.edge_rows(g, uv[:, ::-1], method=method, threads=3)
        np.testing.assert_array_equal(back, want, err_msg=method + " reversed")
    glob = oracle_mod.global_counts(g, want)
    np.testing.assert_array_equal(
        glob, BF.global_instances(n, [tuple(e) for e in uv.tolist()], g.types, L))


def test_brute_force_many_small(oracle_mod):
    """Wider sweep on very small graphs (n <= 8, L <= 4)."""
    rng = np.random.default_rng(1234)
    for s in range(150):
        n = int(rng.integers(4, 9))
        p = float(rng.uniform(0.2, 1.0))
        L = int(rng.integers(1, 5))
        g = G.random_small_graph(n, p, L, 10_000 + s)
        uv = g.edges()
        if uv.shape[0] == 0:
            continue
        want = BF.per_edge_rows(n, [tuple(e) for e in uv.tolist()], g.types, L)
        got = oracle_mod.edge_rows(g, uv, method="paper", threads=1)
        np.testing.assert_array_equal(got, want, err_msg=f"case {s}")


# --------------------------------------------------------- closed forms

def _untyped(oracle_mod, g):
    return oracle_mod.all_edge_rows(g, method="paper", threads=2)


def _orbit_sum(rows, L, g_id):
    P = L * (L + 1) // 2
    return rows[:, 2 * L + (g_id - 3) * P: 2 * L + (g_id - 2) * P].sum(axis=1)


def test_complete_graph(oracle_mod):
    n = 7
    edges = list(itertools.combinations(range(n), 2))
    types = [0, 0, 1, 2, 2, 2, 1]
    L = 3
    g = graph_from_edges(n, edges, types, L)
    rows = oracle_mod.all_edge_rows(g, threads=2)
    idx = BF.column_index(L)
    for q, (i, j) in enumerate(g.edges()):
        c = np.bincount([types[k] for k in range(n) if k not in (i, j)], minlength=L)
        want = {}
        for t in range(L):
            want[f"tri[{t}]"] = c[t]
            for u in range(t, L):
                want[f"g12[{t},{u}]"] = c[t] * (c[t] - 1) // 2 if t == u else c[t] * c[u]
        expect = np.zeros(rows.shape[1], dtype=np.uint64)
        for k, v in want.items():
            expect[idx[k]] = v
        np.testing.assert_array_equal(rows[q], expect)


def test_complete_bipartite(oracle_mod):
    a, b = 4, 5
    edges = [(x, a + y) for x in range(a) for y in range(b)]
    g = graph_from_edges(a + b, edges, [0] * (a + b), 1)
    rows = _untyped(oracle_mod, g)
    for r in rows:
        assert r[0] == 0 and r[1] == a + b - 2
    assert (_orbit_sum(rows, 1, 6) == (a - 1) * (b - 1)).all()
    assert (_orbit_sum(rows, 1, 5) == (a - 1) * (a - 2) // 2 + (b - 1) * (b - 2) // 2).all()
    for gid in (3, 4, 7, 8, 9, 10, 11, 12):
        assert (_orbit_sum(rows, 1, gid) == 0).all()


@pytest.mark.parametrize("n", [4, 5, 9])
def test_cycle(oracle_mod, n):
    edges = [(x, (x + 1) % n) for x in range(n)]
    g = graph_from_edges(n, edges, [0] * n, 1)
    rows = _untyped(oracle_mod, g)
    assert (rows[:, 1] == 2).all()
    if n == 4:
        assert (_orbit_sum(rows, 1, 6) == 1).all()
        others = (3, 4)
    else:
        assert (_orbit_sum(rows, 1, 3) == 2).all()
        assert (_orbit_sum(rows, 1, 4) == 1).all()
        others = (6,)
    for gid in others + (5, 7, 8, 9, 10, 11, 12):
        assert (_orbit_sum(rows, 1, gid) == 0).all()


def test_star(oracle_mod):
    n = 8
    g = graph_from_edges(n, [(0, x) for x in range(1, n)], [0] * n, 1)
    rows = _untyped(oracle_mod, g)
    assert (rows[:, 1] == n - 2).all()
    assert (_orbit_sum(rows, 1, 5) == (n - 2) * (n - 3) // 2).all()


def test_petersen(oracle_mod):
    outer = [(x, (x + 1) % 5) for x in range(5)]
    spokes = [(x, x + 5) for x in range(5)]
    inner = [(5 + x, 5 + (x + 2) % 5) for x in range(5)]
    g = graph_from_edges(10, outer + spokes + inner, [0] * 10, 1)
    rows = _untyped(oracle_mod, g)
    assert rows.shape[0] == 15
    assert rows[:, 0].sum() == 0 and rows[:, 1].sum() == 60
    sums = {gid: int(_orbit_sum(rows, 1, gid).sum()) for gid in range(3, 13)}
    assert sums == {3: 120, 4: 60, 5: 30, 6: 0, 7: 0, 8: 0, 9: 0, 10: 0, 11: 0, 12: 0}
    glob = oracle_mod.global_counts(g, rows)
    # L=1 layout: h0, h1, h2, h3..h8 one entry each
    assert glob.tolist() == [15, 30, 0, 60, 10, 0, 0, 0, 0]


# ----------------------------------------------------------- invariants

def _collapse(g):
    return G.Graph(g.row_ptr, g.col, np.zeros_like(g.types), 1, g.name + "_L1")


@pytest.fixture(scope="module")
def er_small():
    return G.er_graph(300, 9.0, 4, seed=7)


@pytest.fixture(scope="module")
def cl_small():
    return G.chung_lu_typed(3000, 12.0, 2.1, 300.0, 3, type_probs=G.zipf_probs(3, 1.2),
                            homophily=0.6, seed=3)


@pytest.mark.parametrize("which", ["er_small", "cl_small"])
def test_typed_sums_equal_untyped(oracle_mod, request, which):
    """Prop. 1: the typed counts of a graphlet sum to its untyped count."""
    g = request.getfixturevalue(which)
    rows = oracle_mod.all_edge_rows(g, threads=4)
    un = oracle_mod.all_edge_rows(_collapse(g), threads=4)
    L = g.L
    assert (rows[:, :L].sum(axis=1) == un[:, 0]).all()
    assert (rows[:, L:2 * L].sum(axis=1) == un[:, 1]).all()
    for gid in range(3, 13):
        assert (_orbit_sum(rows, L, gid) == _orbit_sum(un, 1, gid)).all()


@pytest.mark.parametrize("which", ["er_small", "cl_small"])
def test_degree_identity_and_lemma_sums(oracle_mod, request, which):
    g = request.getfixturevalue(which)
    L = g.L
    rows = oracle_mod.all_edge_rows(g, threads=4).astype(np.int64)
    uv = g.edges()
    d = g.degrees()
    tri = rows[:, :L].sum(axis=1)
    p3 = rows[:, L:2 * L].sum(axis=1)
    # corrected Property prop:1 (S_i excludes j, S_j excludes i)
    assert (2 * tri + p3 == d[uv[:, 0]] + d[uv[:, 1]] - 2).all()
    Si = d[uv[:, 0]] - 1 - tri
    Sj = d[uv[:, 1]] - 1 - tri
    o = {gid: _orbit_sum(rows, L, gid).astype(np.int64) for gid in range(3, 13)}
    assert (o[4] + o[6] == Si * Sj).all()                               # Lemma 1
    assert (o[5] + o[7] == Si * (Si - 1) // 2 + Sj * (Sj - 1) // 2).all()  # Lemma 2
    assert (o[9] + o[10] == tri * (Si + Sj)).all()                       # Lemma 3
    assert (o[11] + o[12] == tri * (tri - 1) // 2).all()                 # Lemma 4


def test_definition_matches_paper_algorithm(oracle_mod, cl_small):
    a = oracle_mod.all_edge_rows(cl_small, method="paper", threads=4)
    b = oracle_mod.all_edge_rows(cl_small, method="definition", threads=4)
    np.testing.assert_array_equal(a, b)


def test_relabel_invariance(oracle_mod, er_small):
    g = er_small
    rng = np.random.default_rng(5)
    perm = rng.permutation(g.n)           # new id of old node
    uv = g.edges()
    rows = oracle_mod.edge_rows(g, uv, threads=4)
    nu, nv = perm[uv[:, 0]], perm[uv[:, 1]]
    rp, col = G.csr_from_edges(g.n, nu, nv)
    types = np.empty_like(g.types)
    types[perm] = g.types
    h = G.Graph(rp, col, types, g.L, "relabelled")
    rows2 = oracle_mod.edge_rows(h, np.stack([nu, nv], axis=1), threads=4)
    np.testing.assert_array_equal(rows, rows2)


def test_type_permutation_equivariance(oracle_mod, er_small):
    g = er_small
    L = g.L
    sigma = np.array([2, 0, 3, 1])
    h = G.Graph(g.row_ptr, g.col, sigma[g.types].astype(np.uint8), L, "perm")
    a = oracle_mod.all_edge_rows(g, threads=4)
    b = oracle_mod.all_edge_rows(h, threads=4)
    idx = BF.column_index(L)
    for t in range(L):
        np.testing.assert_array_equal(a[:, idx[f"tri[{t}]"]], b[:, idx[f"tri[{sigma[t]}]"]])
        np.testing.assert_array_equal(a[:, idx[f"path3[{t}]"]], b[:, idx[f"path3[{sigma[t]}]"]])
        for u in range(t, L):
            x, y = sorted((sigma[t], sigma[u]))
            for gid in range(3, 13):
                np.testing.assert_array_equal(a[:, idx[f"g{gid}[{t},{u}]"]],
                                              b[:, idx[f"g{gid}[{x},{y}]"]])


def test_global_is_edge_sum_over_edge_count(oracle_mod, cl_small):
    """Problem 2: per-edge sums are |E(H)| times the global count."""
    g = cl_small
    rows = oracle_mod.all_edge_rows(g, threads=4)
    glob = oracle_mod.global_counts(g, rows)
    un_rows = oracle_mod.all_edge_rows(_collapse(g), threads=4)
    un = oracle_mod.global_counts(_collapse(g), un_rows)
    L = g.L
    n2, n3, n4 = len(BF.multisets(L, 2)), len(BF.multisets(L, 3)), len(BF.multisets(L, 4))
    blocks = [glob[:n2], glob[n2:n2 + n3], glob[n2 + n3:n2 + 2 * n3]] + [
        glob[n2 + 2 * n3 + k * n4: n2 + 2 * n3 + (k + 1) * n4] for k in range(6)]
    # typed graphlet counts sum to the untyped global count (Prop. 1)
    assert [int(b.sum()) for b in blocks] == [int(x) for x in un]
    assert un[0] == g.m


def test_oracle_rejects_bad_input(oracle_mod, er_small):
    with pytest.raises(RuntimeError):
        oracle_mod.edge_row(er_small, 0, er_small.n + 5)
