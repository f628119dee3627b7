"""The allocation-free entry point (workspace in the library's static device
scratch) against the ordinary entry point and the oracle, bit for bit, on
two calls in a row, the second with a smaller graph (the scratch keeps the
first call's contents)."""

import numpy as np
import pytest

from gpu_util import to_device
from tg_synth import graphs as G

pytestmark = pytest.mark.gpu


def _noalloc(g):
    import torch

    import paper_2010_14058_amd as P
    from paper_2010_14058_amd import _lib

    rp, col, ty = to_device(g)
    rows = torch.full((g.m, P.row_width(g.L)), -1, dtype=torch.int64, device=rp.device)
    glob = torch.full((P.global_width(g.L),), -1, dtype=torch.int64, device=rp.device)
    stream = torch.cuda.current_stream(rp.device)
    print(f"[gpu] noalloc {g.name}: n={g.n} m={g.m} L={g.L}", flush=True)
    _lib.count_noalloc_raw(rp.data_ptr(), col.data_ptr() if g.nnz else 0, ty.data_ptr(), g.n,
                           g.nnz, g.L, rows.data_ptr(), glob.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    return rows.cpu().numpy().view(np.uint64), glob.cpu().numpy().view(np.uint64)


def _ordinary(g):
    import torch

    import paper_2010_14058_amd as P

    rp, col, ty = to_device(g)
    rows, glob = P.count_typed_graphlets(rp, col, ty, g.L)
    torch.cuda.synchronize()
    return rows.cpu().numpy().view(np.uint64), glob.cpu().numpy().view(np.uint64)


def test_noalloc_matches_ordinary_entry(oracle_mod):
    big = G.chung_lu_typed(20000, 16.0, 2.1, 3000.0, 5, type_probs=G.zipf_probs(5, 1.2),
                           homophily=0.6, seed=5, name="cl_20k")
    small = G.config_graph(1)
    assert small.m < big.m and small.n < big.n
    for g in (big, small):
        rows, glob = _noalloc(g)
        want_rows, want_glob = _ordinary(g)
        np.testing.assert_array_equal(rows, want_rows)
        np.testing.assert_array_equal(glob, want_glob)
        oracle_rows = oracle_mod.all_edge_rows(g)
        np.testing.assert_array_equal(rows, oracle_rows)
        np.testing.assert_array_equal(glob, oracle_mod.global_counts(g, oracle_rows))
