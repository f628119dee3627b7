"""MI355X typed-graphlet counting (Rossi et al., "Heterogeneous Graphlets").

Per-edge and global counts of typed 2-, 3- and 4-node graphlets, computed by
hand-written HIP kernels for gfx950 behind the C ABI of ``include/tg.h``.
PyTorch only supplies device memory and the stream.
"""

from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (  # noqa: F401
    TGError,
    batch_workspace_bytes,
    get_tuning,
    global_key_describe,
    global_width,
    kernel_sums,
    key_describe,
    last_stats,
    pa_global_key_describe,
    pa_global_width,
    pa_key_describe,
    pa_row_width,
    phase_times,
    row_width,
    set_timing,
    set_tuning,
    workspace_bytes,
)

NO_CONVERGENCE = 12  # tg_status TG_E_NO_CONVERGENCE


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


def count_position_aware(row_ptr, col, types, L: int, *, per_edge: bool = True, out_rows=None,
                         out_global=None, workspace: Workspace | None = None, stream=None):
    """Position-aware typed graphlet counts (Sec. 5) of one graph held in
    device tensors; arguments as for :func:`count_typed_graphlets`.  Returns
    ``(rows [nnz/2, pa_row_width(L)] or None, glob [pa_global_width(L)])``,
    int64 tensors holding the uint64 counts, each edge's row oriented from
    its first to its second endpoint in canonical order."""
    import torch

    dev = row_ptr.device
    if dev.type != "cuda":
        raise ValueError("inputs must be device tensors")
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32 or types.dtype != torch.uint8:
        raise TypeError("row_ptr int64, col int32, types uint8 expected")
    row_ptr, col, types = row_ptr.contiguous(), col.contiguous(), types.contiguous()
    n, nnz = row_ptr.numel() - 1, col.numel()
    W = pa_row_width(L)
    if W == 0:
        raise _lib.TGError(4, "count_position_aware")
    rows = None
    if per_edge:
        rows = out_rows if out_rows is not None else torch.empty((nnz // 2, W), dtype=torch.int64,
                                                                 device=dev)
    glob = out_global if out_global is not None else torch.empty(pa_global_width(L),
                                                                 dtype=torch.int64, device=dev)
    wsb = workspace_bytes(n, nnz, L)
    if wsb == 0:
        raise _lib.TGError(1, "tg_workspace_bytes")
    ws = (workspace or Workspace(dev)).get(wsb)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    _lib.count_position_aware_raw(row_ptr.data_ptr(), col.data_ptr() if nnz else 0,
                                  types.data_ptr(), n, nnz, L,
                                  rows.data_ptr() if rows is not None and rows.numel() else 0,
                                  glob.data_ptr(), ws.data_ptr(), ws.numel(), stream.cuda_stream)
    return rows, glob


def global_offsets(graph_L) -> "np.ndarray":
    """Offsets of the per-graph global vectors (each in its graph's own layout)."""
    import numpy as np

    widths = np.array([global_width(int(x)) for x in range(0, 17)], dtype=np.int64)
    gl = np.asarray(graph_L, dtype=np.int64)
    return np.concatenate([[0], np.cumsum(widths[gl])]).astype(np.int64)


class BatchPlan:
    """Device-resident descriptor of a batch of graphs (disjoint-union CSR)."""

    def __init__(self, row_ptr, col, types, node_ptr, graph_L, L_max: int | None = None):
        import numpy as np
        import torch

        self.row_ptr = row_ptr.contiguous()
        self.col = col.contiguous()
        self.types = types.contiguous()
        dev = self.row_ptr.device
        gl_host = graph_L.cpu().numpy() if hasattr(graph_L, "cpu") else np.asarray(graph_L)
        self.node_ptr = torch.as_tensor(np.asarray(node_ptr.cpu() if hasattr(node_ptr, "cpu")
                                                   else node_ptr, dtype=np.int64)).to(dev)
        self.graph_L = torch.as_tensor(gl_host.astype(np.int32)).to(dev)
        self.goff_host = global_offsets(gl_host)
        self.goff = torch.as_tensor(self.goff_host).to(dev)
        self.G = int(gl_host.shape[0])
        self.L_max = int(L_max if L_max is not None else gl_host.max())
        self.n = self.row_ptr.numel() - 1
        self.nnz = self.col.numel()
        np_host = np.asarray(node_ptr.cpu() if hasattr(node_ptr, "cpu") else node_ptr,
                             dtype=np.int64)
        self.max_graph_nodes = int(np.max(np.diff(np_host))) if self.G else 0


def count_batch(plan: BatchPlan, *, per_edge: bool = False, out_globals=None, out_rows=None,
                workspace: Workspace | None = None, stream=None):
    """Typed graphlet counts of every graph of a batch in one library call.

    Returns ``(globals, rows)``: globals is an int64 tensor holding the
    per-graph uint64 global vectors back to back (graph g at
    ``plan.goff_host[g]``, in its own L layout); rows (optional) holds the
    union's per-edge table in the layout of ``plan.L_max``.
    """
    import torch

    dev = plan.row_ptr.device
    glen = int(plan.goff_host[-1])
    glob = out_globals if out_globals is not None else torch.empty(glen, dtype=torch.int64,
                                                                   device=dev)
    rows = None
    if per_edge:
        rows = out_rows if out_rows is not None else torch.empty(
            (plan.nnz // 2, row_width(plan.L_max)), dtype=torch.int64, device=dev)
    wsb = batch_workspace_bytes(plan.n, plan.nnz, plan.G, plan.L_max)
    if wsb == 0:
        raise _lib.TGError(1, "tg_batch_workspace_bytes")
    ws = (workspace or Workspace(dev)).get(wsb)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    _lib.count_batch_raw(plan.row_ptr.data_ptr(), plan.col.data_ptr() if plan.nnz else 0,
                         plan.types.data_ptr(), plan.n, plan.nnz, plan.node_ptr.data_ptr(),
                         plan.graph_L.data_ptr(), plan.G, plan.L_max, plan.goff.data_ptr(), glen,
                         rows.data_ptr() if rows is not None and rows.numel() else 0,
                         glob.data_ptr(), ws.data_ptr(), ws.numel(), stream.cuda_stream)
    return glob, rows


def count_batch_async(plan: BatchPlan, out_globals, status, workspace, stream, *,
                      out_rows=None, max_graph_nodes: int | None = None) -> None:
    """Enqueue the batch on `stream` with no host synchronisation (so it can
    be recorded into a HIP graph): out_globals (int64 [plan.goff_host[-1]])
    receives the per-graph global vectors and status (device int32 [1]) the
    call's status code, both valid once the stream reaches them.  The
    workspace must already hold at least tg_batch_workspace_bytes (the
    call allocates nothing)."""
    wsb = batch_workspace_bytes(plan.n, plan.nnz, plan.G, plan.L_max)
    ws = workspace.get(wsb)
    _lib.count_batch_async_raw(plan.row_ptr.data_ptr(), plan.col.data_ptr() if plan.nnz else 0,
                               plan.types.data_ptr(), plan.n, plan.nnz, plan.node_ptr.data_ptr(),
                               plan.graph_L.data_ptr(), plan.G, plan.L_max,
                               max_graph_nodes or plan.max_graph_nodes, plan.goff.data_ptr(),
                               int(plan.goff_host[-1]),
                               out_rows.data_ptr() if out_rows is not None else 0,
                               out_globals.data_ptr(), ws.data_ptr(), ws.numel(),
                               status.data_ptr(), stream.cuda_stream)


def edge_list(row_ptr, col, *, workspace: Workspace | None = None, stream=None):
    """Canonical (u < v, lexicographic) edge list of a device CSR: an int64
    tensor [nnz/2, 2], the edges of the per-edge rows in order."""
    import torch

    dev = row_ptr.device
    n, nnz = row_ptr.numel() - 1, col.numel()
    uv = torch.empty((nnz // 2, 2), dtype=torch.int64, device=dev)
    ws = (workspace or Workspace(dev)).get(_lib.load().tg_edge_list_workspace_bytes(n))
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    rc = _lib.load().tg_edge_list(row_ptr.data_ptr(), col.data_ptr() if nnz else 0, n, nnz,
                                  uv.data_ptr() if nnz else 0, ws.data_ptr(), ws.numel(),
                                  stream.cuda_stream)
    if rc:
        raise _lib.TGError(rc, "tg_edge_list")
    return uv


def count_directed(row_ptr, col, dirs, types, L: int, *, per_edge: bool = True,
                   workspace: Workspace | None = None, stream=None):
    """Directed typed 2- and 3-node graphlet counts (Sec. 4.8) of a device
    CSR of the underlying undirected graph with per-slot arc bits ``dirs``
    (uint8, bit 0: u -> col[s], bit 1: col[s] -> u).  Returns ``(rows,
    glob)``: rows int64 [nnz/2, 15L] (uint64 bit patterns; None without
    ``per_edge``) and glob int64 [4L^2 + 64L^3]."""
    import torch

    dev = row_ptr.device
    n, nnz = row_ptr.numel() - 1, col.numel()
    lib = _lib.load()
    W = lib.tg_directed_row_width(L)
    G = lib.tg_directed_global_width(L)
    if W == 0:
        raise _lib.TGError(4, "tg_count_directed")
    rows = torch.empty((nnz // 2, W), dtype=torch.int64, device=dev) if per_edge else None
    glob = torch.empty(G, dtype=torch.int64, device=dev)
    ws = (workspace or Workspace(dev)).get(lib.tg_directed_workspace_bytes(n, nnz, L))
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    rc = lib.tg_count_directed(row_ptr.data_ptr(), col.data_ptr() if nnz else 0,
                               dirs.data_ptr() if nnz else 0, types.data_ptr() if n else 0, n,
                               nnz, L, rows.data_ptr() if (rows is not None and nnz) else 0,
                               glob.data_ptr(), ws.data_ptr(), ws.numel(), stream.cuda_stream)
    if rc:
        raise _lib.TGError(rc, "tg_count_directed")
    return rows, glob


def graphlet_weights(rows, edge_uv, types, L: int, graphlet: int, types_sorted, *, stream=None):
    """W_e of Alg. 5 for every edge: the instances of the typed graphlet
    (graphlet id 0..8, sorted type multiset) that contain it, read off the
    per-edge rows (``count_typed_graphlets``) with ``edge_list``'s edges.
    Returns a device int64 tensor [m] holding uint64 counts."""
    import torch

    dev = rows.device
    rows = rows.contiguous()
    m = rows.shape[0]
    if rows.dim() != 2 or rows.shape[1] != row_width(L) or tuple(edge_uv.shape) != (m, 2):
        raise ValueError("rows must be [m, row_width(L)] and edge_uv [m, 2]")
    ms = (ctypes.c_int32 * 4)(*([int(t) for t in types_sorted] + [0] * (4 - len(types_sorted))))
    w = torch.empty(m, dtype=torch.int64, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    rc = _lib.load().tg_graphlet_weights(rows.data_ptr() if m else 0, m, L,
                                         edge_uv.contiguous().data_ptr() if m else 0,
                                         types.data_ptr() if m else 0, graphlet, ms,
                                         w.data_ptr() if m else 0, stream.cuda_stream)
    if rc:
        raise _lib.TGError(rc, "tg_graphlet_weights")
    return w


def graphlet_embedding(row_ptr, col, weights, dim: int, *, max_iter: int = 0, degree: int = 0,
                       tol: float = 0.0, seed: int = 0, raw: bool = False,
                       workspace: Workspace | None = None, stream=None, check: bool = True):
    """Alg. 5's embedding, per connected component of the typed-graphlet
    graph (Sec. 8.8), of a device CSR graph with per-edge weights (canonical
    edge order): ``(Z float64 [n, dim], eigenvalues float64 [n, dim],
    component int32 [n], iterations)``.  Row r of eigenvalues holds the
    spectrum of the component whose smallest node id is r; component is -1
    for nodes in no instance.  Defaults of 0 take the library's (500
    iterations, degree 10, tolerance 1e-10).  With ``raw`` Z holds the
    eigenvectors themselves instead of Alg. 5's unit-length rows.  With
    ``check`` a non-converged solve raises; else the last Ritz pairs are
    returned."""
    import torch

    dev = row_ptr.device
    n, nnz = row_ptr.numel() - 1, col.numel()
    Z = torch.empty((n, dim), dtype=torch.float64, device=dev)
    ev = torch.empty((n, dim), dtype=torch.float64, device=dev)
    comp = torch.empty(n, dtype=torch.int32, device=dev)
    lib = _lib.load()
    ws = (workspace or Workspace(dev)).get(lib.tg_embedding_workspace_bytes(n, nnz, dim))
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    opts = _lib.EmbedOpts(max_iter, degree, tol, seed, int(raw), 0)
    its = ctypes.c_int32(0)
    rc = lib.tg_graphlet_embedding(row_ptr.data_ptr(), col.data_ptr() if nnz else 0, n, nnz,
                                   weights.data_ptr() if nnz else 0, dim, ctypes.byref(opts),
                                   Z.data_ptr(), ev.data_ptr(), comp.data_ptr(),
                                   ctypes.byref(its), ws.data_ptr(), ws.numel(),
                                   stream.cuda_stream)
    if rc and (check or rc != NO_CONVERGENCE):
        raise _lib.TGError(rc, "tg_graphlet_embedding")
    return Z, ev, comp, int(its.value)


def sparse_rows(rows, L: int, *, workspace: Workspace | None = None, stream=None):
    """Nonzero entries of a dense per-edge table (Sec. 4.6's sparse form).

    rows: device int64 tensor [m, row_width(L)] holding uint64 counts, as
    returned by :func:`count_typed_graphlets`.  Returns device tensors
    ``(edge_off int64 [m+1], keys int16 [nnz], counts int64 [nnz])``: edge e
    owns entries ``edge_off[e]:edge_off[e+1]``; keys are column ids (uint16
    bit patterns, see ``key_describe``), columns ascending within an edge.
    """
    import torch

    dev = rows.device
    rows = rows.contiguous()
    m = rows.shape[0]
    if rows.dim() != 2 or rows.shape[1] != row_width(L):
        raise ValueError("rows must be [m, row_width(L)]")
    off = torch.empty(m + 1, dtype=torch.int64, device=dev)
    ws = (workspace or Workspace(dev)).get(_lib.sparse_workspace_bytes(m))
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    _lib.sparse_offsets_raw(rows.data_ptr() if m else 0, m, L, off.data_ptr(), ws.data_ptr(),
                            ws.numel(), stream.cuda_stream)
    total = int(off[m].item())
    keys = torch.empty(total, dtype=torch.int16, device=dev)
    counts = torch.empty(total, dtype=torch.int64, device=dev)
    if total:
        _lib.sparse_fill_raw(rows.data_ptr(), m, L, off.data_ptr(), keys.data_ptr(),
                             counts.data_ptr(), stream.cuda_stream)
    return off, keys, counts
