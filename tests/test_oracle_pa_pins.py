"""Pins of the oracle's position-aware typed graphlet counts (Sec. 5).

* the position-aware rows of both oracle methods (the definition, and Alg.
  1-3 with role-ordered keys plus Lemmas 1-4 per role) against the
  template brute force, whose roles are read off numbered drawings of the
  graphlets, on random tiny graphs in both edge orientations;
* a hand-worked path;
* summing the roles of every block gives the typed row (a typed graphlet is
  a position-aware one with the type order forgotten, Sec. 5.2), and every
  typed class splits into position-aware ones (P_H >= T_H);
* the global classes against the brute force's instance counts, class by
  class, through the oracle's description of each class;
* the number of classes of each graphlet against Burnside's lemma (type
  assignments up to the graphlet's automorphisms);
* swapping the edge's orientation swaps the i and j blocks and transposes
  the ordered pairs whose roles hang at i and j.
"""

import itertools
import math

import numpy as np
import pytest

import brute_force as BF
from tg_synth import graphs as G


def _graph(n, edges, types, L):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    rp, col = G.csr_from_edges(n, e[:, 0], e[:, 1])
    return G.Graph(rp, col, np.asarray(types, dtype=np.uint8), L, "hand")


def _random_graphs(count, seed0, nmax=10, Lmax=4):
    rng = np.random.default_rng(seed0)
    for s in range(count):
        n = int(rng.integers(4, nmax + 1))
        L = int(rng.integers(1, Lmax + 1))
        p = float(rng.uniform(0.15, 0.9))
        yield G.random_small_graph(n, p, L, seed0 + s)


@pytest.mark.parametrize("chunk", range(4))
def test_pa_rows_match_brute_force(oracle_mod, chunk):
    for g in _random_graphs(40, 5000 + 40 * chunk):
        uv = g.edges()
        for orient in (uv, uv[:, ::-1].copy()):
            want = BF.pa_per_edge_rows(g.n, [tuple(e) for e in orient.tolist()], g.types, g.L)
            for method in ("paper", "definition"):
                got = oracle_mod.pa_edge_rows(g, orient, method)
                np.testing.assert_array_equal(got, want, err_msg=f"{method} n={g.n} L={g.L}")


def test_pa_hand_path(oracle_mod):
    """Path 0-1-2-3 with types (0, 1, 2, 0), L = 3, worked by hand:
    edge (0,1): 1 has the other neighbour 2, which continues to 3: path3 at
    j of type 2, and the 4-path i-j-k-r with (k, r) types (2, 0);
    edge (1,2): 0 hangs at i, 3 at j: one 3-path at each end (types 0, 0)
    and the centre-edge 4-path with (x at i, y at j) = (0, 0);
    edge (2,3): 1 hangs at i and continues to 0: path3 at i of type 1 and
    the 4-path r-k-i-j with (k, r) types (1, 0)."""
    g = _graph(4, [(0, 1), (1, 2), (2, 3)], [0, 1, 2, 0], 3)
    names = oracle_mod.pa_column_names(3)
    rows = oracle_mod.pa_all_edge_rows(g)
    want = [{"path_j[2]": 1, "g3j[2,0]": 1},
            {"path_i[0]": 1, "path_j[0]": 1, "g4[0,0]": 1},
            {"path_i[1]": 1, "g3i[1,0]": 1}]
    for q, w in enumerate(want):
        exp = np.zeros(len(names), dtype=np.uint64)
        for k, v in w.items():
            exp[names.index(k)] = v
        np.testing.assert_array_equal(rows[q], exp)


def _fold(pa_row, L):
    """Typed row from a position-aware row: roles summed per block."""
    P = L * (L + 1) // 2
    idx = BF.pa_column_index(L)
    out = np.zeros(2 * L + 10 * P, dtype=np.uint64)
    col = BF.column_index(L)
    for t in range(L):
        out[col[f"tri[{t}]"]] = pa_row[idx[f"tri[{t}]"]]
        out[col[f"path3[{t}]"]] = pa_row[idx[f"path_i[{t}]"]] + pa_row[idx[f"path_j[{t}]"]]
    groups = {3: ["g3i", "g3j"], 4: ["g4"], 5: ["g5i", "g5j"], 6: ["g6"], 7: ["g7i", "g7j"],
              8: ["g8"], 9: ["g9i", "g9j"], 10: ["g10i", "g10j"], 11: ["g11"], 12: ["g12"]}
    for orb, blocks in groups.items():
        for t, u in itertools.combinations_with_replacement(range(L), 2):
            v = np.uint64(0)
            for b in blocks:
                if b in BF.PA_PAIR:
                    v += pa_row[idx[f"{b}{{{t},{u}}}"]]
                else:
                    v += pa_row[idx[f"{b}[{t},{u}]"]]
                    if t != u:
                        v += pa_row[idx[f"{b}[{u},{t}]"]]
            out[col[f"g{orb}[{t},{u}]"]] = v
    return out


def test_pa_fold_is_typed_row(oracle_mod):
    for g in list(_random_graphs(30, 7000)) + [G.config_graph(2, scale=0.002)]:
        pa = oracle_mod.pa_all_edge_rows(g)
        typed = oracle_mod.all_edge_rows(g)
        folded = np.stack([_fold(r, g.L) for r in pa]) if len(pa) else typed
        np.testing.assert_array_equal(folded, typed)


def test_pa_global_matches_brute_force(oracle_mod):
    for g in _random_graphs(30, 9000, nmax=9):
        rows = oracle_mod.pa_all_edge_rows(g)
        glob = oracle_mod.pa_global_counts(g, rows)
        want = BF.pa_global_instances(g.n, [tuple(e) for e in g.edges().tolist()], g.types, g.L)
        got = {}
        for idx in np.nonzero(glob)[0]:
            h, lab = oracle_mod.pa_global_describe(g.L, int(idx))
            key = BF.pa_class_key(h, lab, g.L)
            assert key not in got
            got[key] = int(glob[idx])
        assert got == want


def _burnside(L):
    """Classes of each graphlet: type assignments up to its automorphisms."""
    P = L * (L + 1) // 2
    return [P, L * P, math.comb(L + 2, 3), (L ** 4 + L ** 2) // 2, L * math.comb(L + 2, 3),
            (L ** 4 + 2 * L ** 3 + 3 * L ** 2 + 2 * L) // 8, L * L * P, P * P,
            math.comb(L + 3, 4)]


@pytest.mark.parametrize("L", [1, 2, 3, 5, 7])
def test_pa_class_counts_burnside(oracle_mod, L):
    counts = [0] * 9
    W = oracle_mod.pa_global_width(L)
    seen = set()
    for idx in range(W):
        h, lab = oracle_mod.pa_global_describe(L, idx)
        counts[h] += 1
        key = BF.pa_class_key(h, lab, L)
        assert key not in seen  # every class listed once
        seen.add(key)
    assert counts == _burnside(L)
    assert W == sum(_burnside(L))


def _swap_orientation(row, L):
    idx = BF.pa_column_index(L)
    out = np.zeros_like(row)
    swap = {"path_i": "path_j", "g3i": "g3j", "g5i": "g5j", "g7i": "g7j", "g9i": "g9j",
            "g10i": "g10j"}
    swap.update({v: k for k, v in swap.items()})
    for name, q in idx.items():
        b = name.split("[")[0].split("{")[0]
        rest = name[len(b):]
        if b in ("g4", "g6"):          # (x at i, y at j) becomes (y, x)
            x, y = rest[1:-1].split(",")
            out[idx[f"{b}[{y},{x}]"]] = row[q]
        else:
            out[idx[swap.get(b, b) + rest]] = row[q]
    return out


def test_pa_orientation_swap(oracle_mod):
    for g in _random_graphs(20, 11000):
        uv = g.edges()
        a = oracle_mod.pa_edge_rows(g, uv)
        b = oracle_mod.pa_edge_rows(g, uv[:, ::-1].copy())
        for q in range(len(uv)):
            np.testing.assert_array_equal(b[q], _swap_orientation(a[q], g.L))


def test_pa_splits_typed_classes(oracle_mod):
    """Every typed graphlet's count is the sum of its position-aware
    classes, so there are at least as many nonzero position-aware classes as
    typed ones (P_H >= T_H), with more when one typed class has two
    position-aware ones."""
    strictly_more = False
    for g in list(_random_graphs(15, 12000)) + [G.config_graph(2, scale=0.002)]:
        pa = oracle_mod.pa_global_counts(g, oracle_mod.pa_all_edge_rows(g))
        typed = oracle_mod.global_counts(g, oracle_mod.all_edge_rows(g))
        r = {2: BF.multisets(g.L, 2), 3: BF.multisets(g.L, 3), 4: BF.multisets(g.L, 4)}
        n2, n3, n4 = len(r[2]), len(r[3]), len(r[4])
        starts = [0, n2, n2 + n3] + [n2 + 2 * n3 + q * n4 for q in range(6)]
        folded = np.zeros_like(typed)
        nz_pa = [0] * 9
        for idx in np.nonzero(pa)[0]:
            h, lab = oracle_mod.pa_global_describe(g.L, int(idx))
            ms = tuple(sorted(lab))
            folded[starts[h] + r[len(ms)].index(ms)] += pa[idx]
            nz_pa[h] += 1
        np.testing.assert_array_equal(folded, typed)
        for h in range(9):
            hi = starts[h + 1] if h < 8 else len(typed)
            nz_t = int(np.count_nonzero(typed[starts[h]:hi]))
            assert nz_pa[h] >= nz_t
            strictly_more |= nz_pa[h] > nz_t
    assert strictly_more
