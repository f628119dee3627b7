"""Full-size parity on sampled edges.

The power-law configuration (1M nodes, 10M edges, L = 5) runs at its full
size in the same call the benchmark times.  The oracle recomputes a sample
of edges one by one (uniform edges plus edges at the highest-degree nodes,
where the heavy paths run); every GPU row must match bit for bit.  Over the
whole output, properties that hold at any size are checked: each row's
3-node counts add up to the endpoint degrees (every other neighbour of an
endpoint closes a triangle or a 3-path), and the GPU's global vector is the
one the oracle derives from the GPU's own rows.

A second graph has a node of degree above 2^16, so its 4-cycle group keeps
32-bit map counts, and its biggest groups are split into target ranges.
"""

import numpy as np
import pytest

from gpu_util import to_device
from tg_synth import graphs as G

pytestmark = pytest.mark.gpu


def sample_edges(g, k, seed, top=8, per_top=24):
    """Indices (lexicographic edge order) of k uniform edges plus edges at
    the top-degree nodes and every edge among them."""
    rng = np.random.default_rng(seed)
    uv = g.edges()
    m = uv.shape[0]
    pick = set(rng.choice(m, size=min(k, m), replace=False).tolist())
    d = g.degrees()
    hubs = np.argsort(-d, kind="stable")[:top]
    for h in hubs:
        inc = np.nonzero((uv[:, 0] == h) | (uv[:, 1] == h))[0]
        pick.update(rng.choice(inc, size=min(per_top, inc.size), replace=False).tolist())
    hs = set(hubs.tolist())
    among = np.nonzero(np.isin(uv[:, 0], hubs) & np.isin(uv[:, 1], hubs))[0]
    pick.update(among.tolist())
    assert all(int(uv[e, 0]) in hs and int(uv[e, 1]) in hs for e in among)
    return np.array(sorted(pick), dtype=np.int64)


def run_and_check(oracle_mod, g, k, seed):
    import torch

    import paper_2010_14058_amd as P

    print(f"[gpu] {g.name}: n={g.n} m={g.m} L={g.L}", flush=True)
    rp, col, ty = to_device(g)
    ws = P.Workspace(rp.device)
    rows, glob = P.count_typed_graphlets(rp, col, ty, g.L, workspace=ws)
    torch.cuda.synchronize()
    idx = sample_edges(g, k, seed)
    got = rows.index_select(0, torch.from_numpy(idx).to(rows.device)).cpu().numpy().view(np.uint64)
    uv = g.edges()
    want = oracle_mod.edge_rows(g, uv[idx], method="paper")
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        e, c = bad[0]
        names = oracle_mod.column_names(g.L)
        raise AssertionError(f"{g.name}: {len(bad)} mismatches; first edge {uv[idx[e]].tolist()} "
                             f"col {names[c]} gpu={got[e, c]} oracle={want[e, c]}")
    glob_h = glob.cpu().numpy().view(np.uint64)
    full = rows.cpu().numpy().view(np.uint64)
    del rows
    L = g.L
    d = g.degrees().astype(np.uint64)
    three = 2 * full[:, :L].sum(axis=1) + full[:, L:2 * L].sum(axis=1)
    np.testing.assert_array_equal(three, d[uv[:, 0]] + d[uv[:, 1]] - 2)
    np.testing.assert_array_equal(glob_h, oracle_mod.global_counts(g, full))
    return idx.size


def test_config2_full_size_sampled(oracle_mod):
    g = G.config_graph(2)
    assert g.n == 1_000_000 and g.L == 5
    checked = run_and_check(oracle_mod, g, k=300, seed=11)
    assert checked >= 300


def collapsed_rows(rows, L):
    """Typed rows [m, 2L + 10P] summed over the types of each column block:
    the untyped row [m, 12] (Prop. 1), computed on the device in chunks."""
    import torch

    P = L * (L + 1) // 2
    out = torch.empty((rows.shape[0], 12), dtype=torch.int64, device=rows.device)
    step = 1 << 21
    for a in range(0, rows.shape[0], step):
        r = rows[a:a + step]
        out[a:a + step, 0] = r[:, :L].sum(dim=1)
        out[a:a + step, 1] = r[:, L:2 * L].sum(dim=1)
        out[a:a + step, 2:] = r[:, 2 * L:].reshape(r.shape[0], 10, P).sum(dim=2)
    return out


def test_config3_full_size_sampled(oracle_mod):
    """The tripartite configuration (1.25M nodes, 20.4M edges, L = 3) at full
    size: sampled rows against the oracle (uniform edges, edges at the top
    hubs and at nodes of super-hub degree beyond the super-hub cap, which are
    probed by binary search), the corrected `prop:1` on every row, the
    global vector against the oracle's from the GPU rows, and an untyped
    (L = 1) run equal to the typed rows summed over types (Prop. 1)."""
    import torch

    import paper_2010_14058_amd as P

    g = G.config_graph(3)
    assert g.n == 1_250_000 and g.L == 3
    print(f"[gpu] {g.name}: n={g.n} m={g.m} L={g.L}", flush=True)
    rp, col, ty = to_device(g)
    ws = P.Workspace(rp.device)
    rows, glob = P.count_typed_graphlets(rp, col, ty, g.L, workspace=ws)
    torch.cuda.synchronize()
    st = P.last_stats()
    d = g.degrees()
    sh_deg = P.get_tuning()["sh_deg"]
    assert st["superhub_candidates"] == int(np.sum(d >= sh_deg)), st
    assert st["superhub_candidates"] > st["superhubs"], st
    # internal rank order is (degree, id): the super-hubs are the top ranks,
    # the remaining nodes of super-hub degree are the lowest-ranked of them
    cand = np.nonzero(d >= sh_deg)[0]
    cand = cand[np.lexsort((cand, d[cand]))]
    overflow = cand[: cand.size - st["superhubs"]]
    uv = g.edges()
    rng = np.random.default_rng(17)
    idx = set(sample_edges(g, 300, 13).tolist())
    for h in overflow[rng.choice(overflow.size, size=min(6, overflow.size), replace=False)]:
        inc = np.nonzero((uv[:, 0] == h) | (uv[:, 1] == h))[0]
        idx.update(rng.choice(inc, size=min(12, inc.size), replace=False).tolist())
    idx = np.array(sorted(idx), dtype=np.int64)
    got = rows.index_select(0, torch.from_numpy(idx).to(rows.device)).cpu().numpy().view(np.uint64)
    want = oracle_mod.edge_rows(g, uv[idx], method="paper")
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        e, c = bad[0]
        names = oracle_mod.column_names(g.L)
        raise AssertionError(f"{g.name}: {len(bad)} mismatches; first edge {uv[idx[e]].tolist()} "
                             f"col {names[c]} gpu={got[e, c]} oracle={want[e, c]}")
    L = g.L
    # corrected prop:1 on every row, on the device
    dd = torch.from_numpy(d.astype(np.int64)).to(rows.device)
    ui = torch.from_numpy(uv[:, 0]).to(rows.device)
    vi = torch.from_numpy(uv[:, 1]).to(rows.device)
    three = 2 * rows[:, :L].sum(dim=1) + rows[:, L:2 * L].sum(dim=1)
    assert torch.equal(three, dd[ui] + dd[vi] - 2)
    # untyped run = typed rows summed over types
    ty0 = torch.zeros_like(ty)
    rows1, glob1 = P.count_typed_graphlets(rp, col, ty0, 1, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(rows1, collapsed_rows(rows, L))
    del rows1, ty0, three
    glob_h = glob.cpu().numpy().view(np.uint64)
    full = rows.cpu().numpy().view(np.uint64)
    del rows
    np.testing.assert_array_equal(glob_h, oracle_mod.global_counts(g, full))
    print(f"[gpu] {g.name}: {idx.size} sampled rows identical, "
          f"{overflow.size} nodes of super-hub degree without a bitmap", flush=True)


def test_degree_above_16_bits(oracle_mod):
    """A hub of degree 70000 over random leaf edges (and a second hub sharing
    a third of its leaves): the hub's 4-cycle group has more than 2^16
    items and more wedges than one task takes."""
    rng = np.random.default_rng(5)
    leaves = 70_000
    n = leaves + 2
    a = [np.zeros(leaves, np.int64), np.full(leaves // 3, 1, np.int64)]
    b = [np.arange(2, n, dtype=np.int64), rng.choice(np.arange(2, n), leaves // 3, replace=False)]
    extra = rng.integers(2, n, size=(200_000, 2))
    extra = extra[extra[:, 0] != extra[:, 1]]
    u = np.concatenate(a + [extra[:, 0], np.array([0])])
    v = np.concatenate(b + [extra[:, 1], np.array([1])])
    e = np.unique(np.sort(np.stack([u, v], 1), axis=1), axis=0)
    rp, col = G.csr_from_edges(n, e[:, 0], e[:, 1])
    types = rng.integers(0, 4, size=n).astype(np.uint8)
    g = G.Graph(rp, col, types, 4, "hub70k")
    assert g.degrees().max() > 65535
    run_and_check(oracle_mod, g, k=200, seed=3)
    import paper_2010_14058_amd as P

    st = P.last_stats()
    assert st["heavy_wedges_pass_a"] > 1 << 18, st
