"""GPU parity of the position-aware counts (Sec. 5) with the oracle, bit for
bit: rows and global classes on hand graphs, random small graphs, the
small ER configuration in full, the power-law and tripartite
configurations at reduced scale, graphs that take the heavy paths, L = 1
and L = 16, and empty graphs.  Every run also checks that folding the
roles of each block gives the typed row of the ordinary entry point.  At
full size (the 1M-node power-law graph) sampled rows are checked against
the oracle, and the fold of every row and of the global classes against
the typed counts."""

import json
import os

import numpy as np
import pytest

import brute_force as BF
from gpu_util import to_device
from tg_synth import graphs as G

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def fold_index(L):
    """Typed column of every position-aware column (device-side fold)."""
    pa = BF.pa_column_index(L)
    col = BF.column_index(L)
    out = np.zeros(len(pa), dtype=np.int64)
    orb = {"g3i": 3, "g3j": 3, "g4": 4, "g5i": 5, "g5j": 5, "g6": 6, "g7i": 7, "g7j": 7, "g8": 8,
           "g9i": 9, "g9j": 9, "g10i": 10, "g10j": 10, "g11": 11, "g12": 12}
    for name, q in pa.items():
        b = name.split("[")[0].split("{")[0]
        keys = [int(x) for x in name[len(b) + 1:-1].split(",")]
        if b == "tri":
            out[q] = col[f"tri[{keys[0]}]"]
        elif b in ("path_i", "path_j"):
            out[q] = col[f"path3[{keys[0]}]"]
        else:
            t, u = sorted(keys)
            out[q] = col[f"g{orb[b]}[{t},{u}]"]
    return out


def fold_rows(rows, L):
    import torch

    idx = torch.from_numpy(fold_index(L)).to(rows.device)
    W = 2 * L + 10 * (L * (L + 1) // 2)
    out = torch.zeros((rows.shape[0], W), dtype=torch.int64, device=rows.device)
    step = 1 << 20
    for a in range(0, rows.shape[0], step):
        out[a:a + step].index_add_(1, idx, rows[a:a + step])
    return out


def run_pa(g):
    import torch

    import paper_2010_14058_amd as P

    print(f"[gpu] position-aware {g.name}: n={g.n} m={g.m} L={g.L}", flush=True)
    rp, col, ty = to_device(g)
    ws = P.Workspace(rp.device)
    rows, glob = P.count_position_aware(rp, col, ty, g.L, workspace=ws)
    trows, tglob = P.count_typed_graphlets(rp, col, ty, g.L, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(fold_rows(rows, g.L), trows)
    return rows.cpu().numpy().view(np.uint64), glob.cpu().numpy().view(np.uint64)


def check(oracle_mod, g):
    rows, glob = run_pa(g)
    want = oracle_mod.pa_all_edge_rows(g)
    if not np.array_equal(rows, want):
        bad = np.argwhere(rows != want)
        e, c = bad[0]
        names = oracle_mod.pa_column_names(g.L)
        raise AssertionError(f"{g.name}: {len(bad)} mismatches; first edge {g.edges()[e].tolist()} "
                             f"col {names[c]} gpu={rows[e, c]} oracle={want[e, c]}")
    np.testing.assert_array_equal(glob, oracle_mod.pa_global_counts(g, want))


def _graph(n, edges, types, L, name):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    rp, col = G.csr_from_edges(n, e[:, 0], e[:, 1])
    return G.Graph(rp, col, np.asarray(types, dtype=np.uint8), L, name)


def test_pa_hand_and_random(oracle_mod):
    with open(os.path.join(HERE, "golden", "hand_graphs.json")) as f:
        for c in json.load(f)["graphs"]:
            check(oracle_mod, _graph(c["n"], c["edges"], c["types"], c["L"], c["name"].split()[0]))
    rng = np.random.default_rng(77)
    for s in range(25):
        g = G.random_small_graph(int(rng.integers(4, 50)), float(rng.uniform(0.05, 0.9)),
                                 int(rng.integers(1, 6)), 3000 + s)
        check(oracle_mod, g)


def test_pa_configurations_scaled(oracle_mod):
    check(oracle_mod, G.config_graph(1))
    check(oracle_mod, G.config_graph(2, scale=0.01))
    check(oracle_mod, G.config_graph(3, scale=0.005))


def test_pa_heavy_paths_and_L_extremes(oracle_mod):
    g = G.chung_lu_typed(20000, 16.0, 2.1, 3000.0, 5, type_probs=G.zipf_probs(5, 1.2),
                         homophily=0.6, seed=5, name="cl_20k")
    check(oracle_mod, g)
    check(oracle_mod, G.chung_lu_typed(800, 10.0, 2.1, 120.0, 16, seed=3, name="cl_L16"))
    check(oracle_mod, G.chung_lu_typed(800, 10.0, 2.1, 120.0, 1, seed=3, name="cl_L1"))


def test_pa_empty_graph():
    import torch

    import paper_2010_14058_amd as P

    g = _graph(5, np.zeros((0, 2), dtype=np.int64), [0, 1, 0, 1, 0], 2, "empty")
    rp, col, ty = to_device(g)
    rows, glob = P.count_position_aware(rp, col, ty, 2)
    torch.cuda.synchronize()
    assert rows.shape == (0, P.pa_row_width(2))
    assert not glob.cpu().numpy().any()


def test_pa_full_size_power_law(oracle_mod):
    """The 1M-node power-law graph: sampled rows against the oracle, every
    row folded onto the typed row, and the global classes folded onto the
    typed global counts."""
    import torch

    import paper_2010_14058_amd as P

    g = G.config_graph(2)
    print(f"[gpu] position-aware {g.name}: n={g.n} m={g.m} L={g.L}", flush=True)
    rp, col, ty = to_device(g)
    ws = P.Workspace(rp.device)
    rows, glob = P.count_position_aware(rp, col, ty, g.L, workspace=ws)
    torch.cuda.synchronize()
    uv = g.edges()
    rng = np.random.default_rng(31)
    idx = set(rng.choice(g.m, size=200, replace=False).tolist())
    d = g.degrees()
    for h in np.argsort(-d, kind="stable")[:6]:
        inc = np.nonzero((uv[:, 0] == h) | (uv[:, 1] == h))[0]
        idx.update(rng.choice(inc, size=min(12, inc.size), replace=False).tolist())
    idx = np.array(sorted(idx), dtype=np.int64)
    got = rows.index_select(0, torch.from_numpy(idx).to(rows.device)).cpu().numpy().view(np.uint64)
    want = oracle_mod.pa_edge_rows(g, uv[idx])
    np.testing.assert_array_equal(got, want)
    folded = fold_rows(rows, g.L)
    del rows
    trows, tglob = P.count_typed_graphlets(rp, col, ty, g.L, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(folded, trows)
    del folded, trows
    # global classes folded by type multiset onto the typed global counts
    pa = glob.cpu().numpy().view(np.uint64)
    typed = tglob.cpu().numpy().view(np.uint64)
    L = g.L
    r = {k: BF.multisets(L, k) for k in (2, 3, 4)}
    n2, n3, n4 = len(r[2]), len(r[3]), len(r[4])
    starts = [0, n2, n2 + n3] + [n2 + 2 * n3 + q * n4 for q in range(6)]
    fold = np.zeros_like(typed)
    for q in np.nonzero(pa)[0]:
        h, lab = P.pa_global_key_describe(L, int(q))
        ms = tuple(sorted(lab))
        fold[starts[h] + r[len(ms)].index(ms)] += pa[q]
    np.testing.assert_array_equal(fold, typed)
