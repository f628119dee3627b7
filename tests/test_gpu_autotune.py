"""The autotuner on the GPU: a small search over the degree buckets and the
task size on a power-law graph, where every setting's counts must agree
(the tuner checks each call's digest) and the tuned counts equal the
oracle's."""

import numpy as np
import pytest

from gpu_util import to_device
from tg_synth import graphs as G

pytestmark = pytest.mark.gpu


def test_tune_small_space(oracle_mod):
    import torch

    import paper_2010_14058_amd as P
    from paper_2010_14058_amd import autotune as AT

    g = G.config_graph(2, scale=0.01)
    print(f"[gpu] autotune on {g.name}: n={g.n} m={g.m}", flush=True)
    rp, col, ty = to_device(g)
    ws = P.Workspace(rp.device)
    rows = torch.empty((g.m, P.row_width(g.L)), dtype=torch.int64, device=rp.device)
    glob = torch.empty(P.global_width(g.L), dtype=torch.int64, device=rp.device)

    def run():
        P.count_typed_graphlets(rp, col, ty, g.L, out_rows=rows, out_global=glob, workspace=ws)
        torch.cuda.synchronize()
        return AT.digest_of(glob, rows)

    base = P.get_tuning()
    try:
        space = {"light_wedges": [512, 32], "edge_deg": [1024, 8], "task_wedges": [1 << 18, 256]}
        res = AT.tune(run, space, repeats=1, rounds=1, log=None)
        assert set(res.best) == set(space)
        assert all(res.best[k] in v for k, v in space.items())
        assert len(res.trials) == 4
        run()
        want = oracle_mod.all_edge_rows(g, threads=8)
        np.testing.assert_array_equal(rows.cpu().numpy().view(np.uint64), want)
        np.testing.assert_array_equal(glob.cpu().numpy().view(np.uint64),
                                      oracle_mod.global_counts(g, want))
    finally:
        P.set_tuning(**base)
