"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Per-edge rows and global counts must be identical (exact integers).  The
cases cover several tiles and ragged tails of every kernel: tiny graphs,
the small Erdos-Renyi configuration in full, scaled-down power-law and
tripartite configurations in full, graphs that route work to the heavy
4-cycle and heavy clique paths, L = 1 and L = 16, empty graphs, and the
input checks.
"""

import json
import os

import numpy as np
import pytest

import brute_force as BF
from gpu_util import run_gpu, to_device
from tg_synth import graphs as G

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def check(oracle_mod, g, method="paper", threads=8):
    rows, glob = run_gpu(g)
    want = oracle_mod.all_edge_rows(g, method=method, threads=threads)
    assert rows.shape == want.shape
    if not np.array_equal(rows, want):
        bad = np.argwhere(rows != want)
        names = oracle_mod.column_names(g.L)
        uv = g.edges()
        e, c = bad[0]
        raise AssertionError(
            f"{g.name}: {len(bad)} mismatches; first edge {uv[e].tolist()} col {names[c]} "
            f"gpu={rows[e, c]} oracle={want[e, c]}")
    np.testing.assert_array_equal(glob, oracle_mod.global_counts(g, want))
    return rows, glob


def graph_from_edges(n, edges, types, L, name="hand"):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    rp, col = G.csr_from_edges(n, e[:, 0], e[:, 1])
    return G.Graph(rp, col, np.asarray(types, dtype=np.uint8), L, name)


def test_hand_graphs(oracle_mod):
    with open(os.path.join(HERE, "golden", "hand_graphs.json")) as f:
        cases = json.load(f)["graphs"]
    for c in cases:
        g = graph_from_edges(c["n"], c["edges"], c["types"], c["L"], c["name"].split(" ")[0])
        check(oracle_mod, g)


def test_random_small(oracle_mod):
    rng = np.random.default_rng(2024)
    for s in range(40):
        n = int(rng.integers(4, 60))
        L = int(rng.integers(1, 6))
        p = float(rng.uniform(0.05, 0.9))
        g = G.random_small_graph(n, p, L, 500 + s)
        check(oracle_mod, g)


def test_brute_force_direct():
    """A few tiny graphs straight against the template brute force."""
    for s in range(10):
        g = G.random_small_graph(9, 0.5, 3, 900 + s)
        if g.m == 0:
            continue
        rows, glob = run_gpu(g)
        uv = [tuple(e) for e in g.edges().tolist()]
        np.testing.assert_array_equal(rows, BF.per_edge_rows(g.n, uv, g.types, g.L))
        np.testing.assert_array_equal(glob, BF.global_instances(g.n, uv, g.types, g.L))


def test_config1_er_full(oracle_mod):
    check(oracle_mod, G.config_graph(1))


def test_config2_scaled_full(oracle_mod):
    check(oracle_mod, G.config_graph(2, scale=0.01))


def test_config3_scaled_full(oracle_mod):
    check(oracle_mod, G.config_graph(3, scale=0.005))


def test_heavy_paths(oracle_mod):
    """Two adjacent hubs sharing 1500 neighbours (both degrees above the
    light clique capacity) plus random leaf edges: heavy edge path and heavy
    4-cycle groups."""
    rng = np.random.default_rng(7)
    hubs = 2
    leaves = 1500
    n = hubs + leaves + 300
    edges = [(0, 1)]
    for x in range(hubs, hubs + leaves):
        edges += [(0, x), (1, x)]
    extra = rng.integers(hubs, n, size=(6000, 2))
    edges += [tuple(e) for e in extra.tolist() if e[0] != e[1]]
    types = rng.integers(0, 3, size=n)
    g = graph_from_edges(n, edges, types, 3, "two_hubs")
    import paper_2010_14058_amd as P

    check(oracle_mod, g)
    st = P.last_stats()
    assert st["heavy_edges"] >= 1 and st["heavy_groups"] >= 1, st


def test_power_law_medium(oracle_mod):
    g = G.chung_lu_typed(20000, 16.0, 2.1, 3000.0, 5, type_probs=G.zipf_probs(5, 1.2),
                         homophily=0.6, seed=5, name="cl_20k")
    check(oracle_mod, g)


@pytest.mark.parametrize("knobs", [dict(sh_max=2), dict(sh_max=0), dict(sh_deg=32)],
                         ids=["two_superhubs", "no_superhubs", "superhub_degree_32"])
def test_superhub_overflow(oracle_mod, knobs):
    """Nodes of super-hub degree without a bitmap: with the super-hub cap at
    2 (or 0) the other nodes of degree >= 1024 are probed by binary search in
    the triangle, clique and gather walks; with the super-hub degree at 32
    most hub-core nodes get bitmaps, and edges joining two super-hubs reach
    the one-wave clique kernel."""
    import paper_2010_14058_amd as P

    old = P.set_tuning(**knobs)
    try:
        g = G.chung_lu_typed(20000, 16.0, 2.1, 3000.0, 5, type_probs=G.zipf_probs(5, 1.2),
                             homophily=0.6, seed=5, name="cl_20k_sh")
        check(oracle_mod, g)
        st = P.last_stats()
        d = g.degrees()
        cap = knobs.get("sh_max", 2048)
        deg = knobs.get("sh_deg", 1024)
        assert st["superhub_candidates"] == int(np.sum(d >= deg)), st
        assert st["superhubs"] == min(cap, st["superhub_candidates"]), st
        if "sh_max" in knobs:
            assert st["superhub_candidates"] > st["superhubs"], st
        else:
            assert st["superhubs"] > 1000, st
    finally:
        P.set_tuning(**old)


def test_max_and_min_L(oracle_mod):
    g16 = G.chung_lu_typed(800, 10.0, 2.1, 120.0, 16, seed=3, name="cl_L16")
    check(oracle_mod, g16)
    g1 = G.chung_lu_typed(800, 10.0, 2.1, 120.0, 1, seed=3, name="cl_L1")
    check(oracle_mod, g1)


def test_no_edges_and_single_edge(oracle_mod):
    g0 = graph_from_edges(5, np.zeros((0, 2), dtype=np.int64), [0, 1, 0, 1, 0], 2, "empty")
    rows, glob = run_gpu(g0)
    assert rows.shape == (0, 2 * 2 + 10 * 3)
    assert not glob.any()
    g1 = graph_from_edges(3, [(0, 2)], [1, 0, 1], 2, "single")
    check(oracle_mod, g1)


def test_global_only_matches(oracle_mod):
    g = G.config_graph(2, scale=0.005)
    rows, glob = run_gpu(g)
    _, glob2 = run_gpu(g, per_edge=False)
    np.testing.assert_array_equal(glob, glob2)


def test_deterministic_and_workspace_reuse():
    import paper_2010_14058_amd as P

    g = G.config_graph(2, scale=0.01)
    ws = P.Workspace()
    a, ga = run_gpu(g, workspace=ws)
    b, gb = run_gpu(g, workspace=ws)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ga, gb)


def _status(g, L=None):
    import torch

    import paper_2010_14058_amd as P

    rp, col, ty = to_device(g)
    try:
        P.count_typed_graphlets(rp, col, ty, L or g.L)
        torch.cuda.synchronize()
    except P.TGError as e:
        return e.code
    return 0


def test_invalid_inputs():
    base = graph_from_edges(4, [(0, 1), (1, 2), (2, 3)], [0, 1, 0, 1], 2, "path")
    assert _status(base) == 0
    # type out of range
    bad_t = G.Graph(base.row_ptr, base.col, np.array([0, 1, 2, 1], np.uint8), 2, "badtype")
    assert _status(bad_t) == 3
    # L out of range
    assert _status(base, L=17) == 4
    # self-loop
    rp = np.array([0, 2, 3, 5, 6], np.int64)
    col = np.array([0, 1, 0, 1, 3, 2], np.int32)
    assert _status(G.Graph(rp, col, base.types, 2, "selfloop")) == 2
    # unsorted row
    rp = np.array([0, 1, 3, 5, 6], np.int64)
    col = np.array([1, 2, 0, 1, 3, 2], np.int32)
    assert _status(G.Graph(rp, col, base.types, 2, "unsorted")) == 2
    # asymmetric (0-1 present one way only, 2-3 both ways)
    rp = np.array([0, 1, 1, 2, 3], np.int64)
    col = np.array([1, 3, 2], np.int32)
    rp2 = np.array([0, 1, 2, 3, 4], np.int64)
    col2 = np.array([1, 2, 3, 2], np.int32)
    assert _status(G.Graph(rp2, col2, base.types, 2, "asym")) == 2
    # asymmetric with as many larger as smaller neighbours (0->1 and 3->2 only)
    rp3 = np.array([0, 1, 1, 1, 2], np.int64)
    col3 = np.array([1, 2], np.int32)
    assert _status(G.Graph(rp3, col3, base.types, 2, "asym2")) == 2
    # odd nnz
    assert _status(G.Graph(rp, col, base.types, 2, "odd")) == 1
    # neighbour id out of range
    rp = np.array([0, 1, 2, 3, 4], np.int64)
    col = np.array([1, 0, 9, 2], np.int32)
    assert _status(G.Graph(rp, col, base.types, 2, "range")) == 2


@pytest.mark.parametrize("knobs", [dict(task_wedges=64, clear_bytes=0),
                                   dict(task_wedges=64, clear_bytes=1 << 20),
                                   dict(range_bytes=512)],
                         ids=["walk_clear", "streamed_clear", "id_ranges"])
def test_split_heavy_tasks(oracle_mod, knobs):
    """Heavy 4-cycle groups split into many target ranges (64 wedges per
    task, or 512 bytes of map entries per task), with map ranges cleared by
    wedge walks or by streaming: the counts must not change."""
    import paper_2010_14058_amd as P

    old = P.set_tuning(**knobs)
    try:
        g = G.chung_lu_typed(20000, 16.0, 2.1, 3000.0, 5, type_probs=G.zipf_probs(5, 1.2),
                             homophily=0.6, seed=5, name="cl_20k_split")
        check(oracle_mod, g)
        assert P.last_stats()["heavy_groups"] >= 1
        check(oracle_mod, G.config_graph(2, scale=0.01))
    finally:
        P.set_tuning(**old)


@pytest.mark.parametrize("knobs", [dict(blk_wedges=1, blk_wedges_b=1),
                                   dict(blk_wedges=4000, blk_wedges_b=4000),
                                   dict(blk_wedges=1, blk_wedges_b=1, blk_bytes="half"),
                                   dict(blk_wedges=1, blk_wedges_b=1, light_wedges=1),
                                   dict(blk_wedges=1, blk_wedges_b=1, blk_task=1024)],
                         ids=["heavy_blocked", "large_blocked", "record_space_cut",
                              "every_group", "small_tasks"])
def test_blocked_groups(oracle_mod, knobs):
    """Heavy 4-cycle groups counted by the blocked path (records per target
    block, LDS block counts into one map per group, emit walk over wedge
    ranges): every heavy group, only the large ones, a record space that
    sends most groups back to the task kernel, every group of two or more
    wedges (more candidates than list slots), and walk tasks of 1024 wedges
    (items spread over several tasks).  Counts must not change; L = 16
    fills the record's four type bits."""
    import paper_2010_14058_amd as P

    g = G.chung_lu_typed(20000, 16.0, 2.1, 3000.0, 5, type_probs=G.zipf_probs(5, 1.2),
                         homophily=0.6, seed=5, name="cl_20k_blocked")
    knobs = dict(knobs)
    if knobs.get("blk_bytes") == "half":
        # records for about half of pass A's heavy wedges: the selection
        # must stop inside the size bins
        old = P.set_tuning(blk_bytes=0)
        run_gpu(g, per_edge=False)
        P.set_tuning(**old)
        knobs["blk_bytes"] = P.last_stats()["heavy_wedges_pass_a"]
    old = P.set_tuning(**knobs)
    try:
        check(oracle_mod, g)
        st = P.last_stats()
        assert st["blocked_groups"] >= 1
        assert st["blocked_wedges_pass_a"] > 0 and st["blocked_wedges_pass_b"] > 0
        assert st["blocked_wedges_pass_a"] <= st["heavy_wedges_pass_a"]
        if "blk_bytes" in knobs:
            assert st["blocked_wedges_pass_a"] <= knobs["blk_bytes"] // 2
            assert st["blocked_wedges_pass_a"] < st["heavy_wedges_pass_a"]
        check(oracle_mod, G.config_graph(2, scale=0.01))
        check(oracle_mod, G.chung_lu_typed(3000, 12.0, 2.1, 800.0, 16, seed=3, name="cl_3k_L16"))
        assert P.last_stats()["blocked_groups"] >= 1
    finally:
        P.set_tuning(**old)


@pytest.mark.parametrize("hub_lds", [0, 64, 65536])
def test_pass_b_hub_targets(oracle_mod, hub_lds):
    """Pass-B targets among the top-ranked ids counted in LDS: off, a hub set
    of a few ids (the boundary inside most target lists) and the largest LDS
    share; counts must not change (L = 5 and L = 16)."""
    import paper_2010_14058_amd as P

    old = P.set_tuning(hub_lds=hub_lds)
    try:
        g = G.chung_lu_typed(20000, 16.0, 2.1, 3000.0, 5, type_probs=G.zipf_probs(5, 1.2),
                             homophily=0.6, seed=5, name="cl_20k_hub")
        check(oracle_mod, g)
        check(oracle_mod, G.chung_lu_typed(3000, 12.0, 2.1, 800.0, 16, seed=3, name="cl_3k_L16"))
    finally:
        P.set_tuning(**old)


@pytest.mark.parametrize("derive_edges", [1, 2, 3, 4])
def test_derive_batching(oracle_mod, derive_edges):
    """The light kernel derives several edges' rows in one wave; every batch
    size gives the same counts (L = 3 and L = 5, heavy edges interleaved)."""
    import paper_2010_14058_amd as P

    old = P.set_tuning(derive_edges=derive_edges)
    try:
        check(oracle_mod, G.config_graph(2, scale=0.005))
        g = G.chung_lu_typed(3000, 12.0, 2.1, 1500.0, 3, seed=9, name="cl_3k_L3")
        check(oracle_mod, g)
    finally:
        P.set_tuning(**old)


@pytest.mark.parametrize("knobs", [dict(light_wedges=1, edge_deg=1),
                                   dict(light_wedges=64, edge_deg=16),
                                   dict(light_wedges=512, edge_deg=1024)],
                         ids=["all_heavy", "small_buckets", "largest_buckets"])
def test_degree_buckets(oracle_mod, knobs):
    """The degree buckets only move 4-cycle groups and edges between the
    one-wave and the workgroup kernels: with every group and edge sent to
    the workgroup kernels, with small buckets and with the largest ones the
    counts are the same (a single graph and a batch)."""
    import paper_2010_14058_amd as P

    old = P.set_tuning(**knobs)
    try:
        g = G.chung_lu_typed(4000, 10.0, 2.1, 600.0, 4, seed=21, name="cl_4k_buckets")
        check(oracle_mod, g)
        st = P.last_stats()
        d = g.degrees()
        uv = g.edges()
        assert st["heavy_edges"] == int(np.sum(np.minimum(d[uv[:, 0]], d[uv[:, 1]]) >
                                               knobs["edge_deg"]))
        check(oracle_mod, G.config_graph(1))
        b = G.batch_graphs(60, seed=4)
        u = b.union
        import torch

        dev = torch.device("cuda:0")
        plan = P.BatchPlan(torch.from_numpy(u.row_ptr).to(dev), torch.from_numpy(u.col).to(dev),
                           torch.from_numpy(u.types).to(dev), b.node_ptr, b.L)
        glob, _ = P.count_batch(plan)
        got = glob.cpu().numpy().view(np.uint64)
        for q in range(b.G):
            gg = b.graph(q)
            want = oracle_mod.global_counts(gg, oracle_mod.all_edge_rows(gg))
            np.testing.assert_array_equal(got[plan.goff_host[q]:plan.goff_host[q + 1]], want)
    finally:
        P.set_tuning(**old)


def test_edge_list():
    """The canonical edge list is the order of the per-edge rows."""
    import torch

    import paper_2010_14058_amd as P

    for g in (G.config_graph(1), G.config_graph(2, scale=0.005),
              graph_from_edges(6, [(0, 5), (1, 2)], [0, 1, 0, 1, 0, 1], 2, "sparse")):
        rp, col, _ = to_device(g)
        uv = P.edge_list(rp, col)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(uv.cpu().numpy(), g.edges())
    # more entries above the diagonal than half the adjacency: refused
    rp = torch.tensor([0, 2, 2, 2], dtype=torch.int64, device="cuda")
    col = torch.tensor([1, 2], dtype=torch.int32, device="cuda")
    with pytest.raises(P.TGError) as e:
        P.edge_list(rp, col)
    assert e.value.code == 2
