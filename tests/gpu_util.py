"""Helpers for the GPU tests: run the HIP library on a tg_synth Graph."""

from __future__ import annotations

import sys

import numpy as np


def device():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda:0")


def to_device(g):
    import torch

    dev = device()
    return (torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(dev),
            torch.from_numpy(np.ascontiguousarray(g.col)).to(dev),
            torch.from_numpy(np.ascontiguousarray(g.types)).to(dev))


def run_gpu(g, per_edge=True, L=None, workspace=None):
    """(rows uint64 [M, W] or None, global uint64 [G]) computed by the library."""
    import torch

    import paper_2010_14058_amd as P

    print(f"[gpu] {g.name}: n={g.n} m={g.m} L={L or g.L}", flush=True)
    sys.stdout.flush()
    rp, col, ty = to_device(g)
    rows, glob = P.count_typed_graphlets(rp, col, ty, L or g.L, per_edge=per_edge,
                                         workspace=workspace)
    torch.cuda.synchronize()
    r = rows.cpu().numpy().view(np.uint64) if rows is not None else None
    return r, glob.cpu().numpy().view(np.uint64)
