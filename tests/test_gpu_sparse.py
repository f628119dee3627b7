"""Sparse per-edge output (Sec. 4.6) against the oracle's dense rows.

The library's sparse form of a dense table must list, for every edge in
canonical order, exactly the nonzero columns of the oracle's row (ascending)
with their counts.
"""

import numpy as np
import pytest

from gpu_util import run_gpu, to_device
from tg_synth import graphs as G

pytestmark = pytest.mark.gpu


def expected_sparse(rows):
    nz = rows != 0
    off = np.concatenate([[0], np.cumsum(nz.sum(axis=1))]).astype(np.int64)
    e, c = np.nonzero(nz)
    return off, c.astype(np.int64), rows[e, c]


def sparse_of(g):
    import torch

    import paper_2010_14058_amd as P

    rp, col, ty = to_device(g)
    rows, _ = P.count_typed_graphlets(rp, col, ty, g.L)
    off, keys, counts = P.sparse_rows(rows, g.L)
    torch.cuda.synchronize()
    return (off.cpu().numpy(), keys.cpu().numpy().view(np.uint16).astype(np.int64),
            counts.cpu().numpy().view(np.uint64))


@pytest.mark.parametrize("name", ["cl_20k", "cl_L16", "config2_small"])
def test_sparse_matches_oracle_nonzeros(oracle_mod, name):
    if name == "cl_20k":
        g = G.chung_lu_typed(20000, 16.0, 2.1, 3000.0, 5, type_probs=G.zipf_probs(5, 1.2),
                             homophily=0.6, seed=5, name=name)
    elif name == "cl_L16":
        g = G.chung_lu_typed(800, 10.0, 2.1, 120.0, 16, seed=3, name=name)
    else:
        g = G.config_graph(2, scale=0.01)
    print(f"[gpu] sparse {g.name}: n={g.n} m={g.m} L={g.L}", flush=True)
    want = oracle_mod.all_edge_rows(g, threads=8)
    off, keys, counts = sparse_of(g)
    w_off, w_keys, w_counts = expected_sparse(want)
    np.testing.assert_array_equal(off, w_off)
    np.testing.assert_array_equal(keys, w_keys)
    np.testing.assert_array_equal(counts, w_counts)


def test_sparse_edge_cases():
    import torch

    import paper_2010_14058_amd as P

    # no edges
    g0 = G.Graph(np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(3, np.uint8), 2, "empty")
    off, keys, counts = sparse_of(g0)
    assert off.tolist() == [0] and keys.size == 0 and counts.size == 0
    # a perfect matching: every row is zero
    n = 10
    u = np.arange(0, n, 2)
    rp, col = G.csr_from_edges(n, u, u + 1)
    g1 = G.Graph(rp, col, np.zeros(n, np.uint8), 3, "matching")
    off, keys, counts = sparse_of(g1)
    assert off.tolist() == [0] * (n // 2 + 1) and keys.size == 0
    # a dense table given directly (rows of arbitrary values)
    L = 2
    W = P.row_width(L)
    rng = np.random.default_rng(0)
    dense = rng.integers(0, 3, size=(37, W)).astype(np.int64)
    dense[5] = 0
    d_off, d_keys, d_counts = P.sparse_rows(torch.from_numpy(dense).to("cuda:0"), L)
    w_off, w_keys, w_counts = expected_sparse(dense.view(np.uint64))
    np.testing.assert_array_equal(d_off.cpu().numpy(), w_off)
    np.testing.assert_array_equal(d_keys.cpu().numpy().astype(np.int64), w_keys)
    np.testing.assert_array_equal(d_counts.cpu().numpy().view(np.uint64), w_counts)
