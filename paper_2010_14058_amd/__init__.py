"""MI355X typed-graphlet counting (Rossi et al., "Heterogeneous Graphlets").

Per-edge and global counts of typed 2-, 3- and 4-node graphlets, computed by
hand-written HIP kernels for gfx950 behind the C ABI of ``include/tg.h``.
PyTorch only supplies device memory and the stream.
"""

from __future__ import annotations

from . import _lib
from ._lib import (  # noqa: F401
    TGError,
    global_key_describe,
    global_width,
    key_describe,
    last_stats,
    phase_times,
    row_width,
    set_timing,
    workspace_bytes,
)


class Workspace:
    """Reusable device workspace (a torch uint8 tensor) grown on demand."""

    def __init__(self, device=None):
        self.device = device
        self.buf = None

    def get(self, nbytes: int):
        import torch

        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device or "cuda")
        return self.buf


def count_typed_graphlets(row_ptr, col, types, L: int, *, per_edge: bool = True,
                          out_rows=None, out_global=None, workspace: Workspace | None = None,
                          stream=None):
    """Typed graphlet counts of one graph held in device tensors.

    row_ptr: int64 [n+1], col: int32 [nnz], types: uint8 [n] on a HIP device.
    Returns ``(rows, glob)``: rows is an int64 tensor [nnz/2, row_width(L)]
    holding the uint64 counts bit for bit (None if ``per_edge`` is False);
    glob is an int64 tensor [global_width(L)].  Rows follow the canonical
    (u < v, lexicographic) edge order.
    """
    import torch

    dev = row_ptr.device
    if dev.type != "cuda":
        raise ValueError("inputs must be device tensors")
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32 or types.dtype != torch.uint8:
        raise TypeError("row_ptr int64, col int32, types uint8 expected")
    row_ptr = row_ptr.contiguous()
    col = col.contiguous()
    types = types.contiguous()
    n = row_ptr.numel() - 1
    nnz = col.numel()
    W = row_width(L)
    G = global_width(L)
    if W == 0:
        raise _lib.TGError(4, "count_typed_graphlets")
    rows = None
    if per_edge:
        rows = out_rows if out_rows is not None else torch.empty((nnz // 2, W), dtype=torch.int64,
                                                                 device=dev)
    glob = out_global if out_global is not None else torch.empty(G, dtype=torch.int64, device=dev)
    wsb = workspace_bytes(n, nnz, L)
    if wsb == 0:
        raise _lib.TGError(1, "tg_workspace_bytes")
    ws = (workspace or Workspace(dev)).get(wsb)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    _lib.count_raw(row_ptr.data_ptr(), col.data_ptr() if nnz else 0, types.data_ptr(), n, nnz, L,
                   rows.data_ptr() if rows is not None and rows.numel() else 0,
                   glob.data_ptr(), ws.data_ptr(), ws.numel(), stream.cuda_stream)
    return rows, glob
