"""ctypes binding of ``libtg.so`` (argument marshalling only).

Every count is computed by the HIP kernels behind the C ABI in
``include/tg.h``; this module only passes device pointers, sizes and the
stream.  It raises if the library has not been built: there is no CPU
fallback.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtg.so")

# Every function the header declares, with its ctypes signature.
_c = ctypes


class GraphDesc(ctypes.Structure):
    """tg_graph_desc"""
    _fields_ = [("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("types", ctypes.c_void_p), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("L", ctypes.c_int32), ("mem", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    """tg_request_info"""
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32),
                ("global_counts", ctypes.c_void_p), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("batch", ctypes.c_int64)]


class EmbedOpts(ctypes.Structure):
    """tg_embed_opts"""
    _fields_ = [("max_iter", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("tol", ctypes.c_double), ("seed", ctypes.c_uint64), ("raw", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


SIGNATURES = {
    "tg_status_str": (_c.c_char_p, [_c.c_int]),
    "tg_row_width": (_c.c_int32, [_c.c_int32]),
    "tg_global_width": (_c.c_int32, [_c.c_int32]),
    "tg_workspace_bytes": (_c.c_size_t, [_c.c_int64, _c.c_int64, _c.c_int32]),
    "tg_count_typed_graphlets": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int64,
                                            _c.c_int64, _c.c_int32, _c.c_void_p, _c.c_void_p,
                                            _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "tg_count_typed_graphlets_noalloc": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p,
                                                    _c.c_int64, _c.c_int64, _c.c_int32,
                                                    _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "tg_batch_workspace_bytes": (_c.c_size_t, [_c.c_int64, _c.c_int64, _c.c_int64, _c.c_int32]),
    "tg_count_batch": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int64,
                                  _c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int32, _c.c_void_p,
                                  _c.c_int64, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_size_t,
                                  _c.c_void_p]),
    "tg_count_batch_async": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int64,
                                        _c.c_int64, _c.c_void_p, _c.c_void_p, _c.c_int64,
                                        _c.c_int32, _c.c_int64, _c.c_void_p, _c.c_int64,
                                        _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_size_t,
                                        _c.c_void_p, _c.c_void_p]),
    "tg_key_describe": (_c.c_int, [_c.c_int32, _c.c_int32, _c.POINTER(_c.c_int32),
                                   _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    "tg_global_key_describe": (_c.c_int, [_c.c_int32, _c.c_int32, _c.POINTER(_c.c_int32),
                                          _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    "tg_set_timing": (None, [_c.c_int32]),
    "tg_phase_times": (_c.c_int32, [_c.POINTER(_c.c_float), _c.POINTER(_c.c_char_p), _c.c_int32]),
    "tg_last_stats": (_c.c_int32, [_c.POINTER(_c.c_int64), _c.c_int32]),
    "tg_set_tuning": (_c.c_int, [_c.c_int32, _c.c_int64]),
    "tg_last_error": (_c.c_char_p, []),
    "tg_edge_list_workspace_bytes": (_c.c_size_t, [_c.c_int64]),
    "tg_edge_list": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int64, _c.c_void_p,
                                _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "tg_sparse_workspace_bytes": (_c.c_size_t, [_c.c_int64]),
    "tg_sparse_offsets": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int32, _c.c_void_p, _c.c_void_p,
                                     _c.c_size_t, _c.c_void_p]),
    "tg_sparse_fill": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int32, _c.c_void_p, _c.c_void_p,
                                  _c.c_void_p, _c.c_void_p]),
    "tg_get_tuning": (_c.c_int64, [_c.c_int32]),
    "tg_server_create": (_c.c_int, [_c.c_void_p, _c.c_size_t, _c.c_int32, _c.c_size_t,
                                    _c.c_int64, _c.c_int64, _c.POINTER(_c.c_void_p)]),
    "tg_server_submit": (_c.c_int, [_c.c_void_p, _c.POINTER(GraphDesc), _c.POINTER(_c.c_int64)]),
    "tg_server_poll": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.POINTER(RequestInfo)]),
    "tg_server_wait": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_double]),
    "tg_server_take_done": (_c.c_int32, [_c.c_void_p, _c.POINTER(_c.c_int64), _c.c_int32,
                                         _c.c_double]),
    "tg_server_release": (_c.c_int, [_c.c_void_p, _c.c_int64]),
    "tg_server_stats": (_c.c_int32, [_c.c_void_p, _c.POINTER(_c.c_int64), _c.c_int32]),
    "tg_server_destroy": (_c.c_int, [_c.c_void_p]),
    "tg_pa_row_width": (_c.c_int32, [_c.c_int32]),
    "tg_pa_global_width": (_c.c_int64, [_c.c_int32]),
    "tg_count_position_aware": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int64,
                                           _c.c_int64, _c.c_int32, _c.c_void_p, _c.c_void_p,
                                           _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "tg_pa_key_describe": (_c.c_int, [_c.c_int32, _c.c_int32, _c.POINTER(_c.c_int32),
                                      _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    "tg_pa_global_key_describe": (_c.c_int, [_c.c_int32, _c.c_int64, _c.POINTER(_c.c_int32),
                                             _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    "tg_kernel_sums": (_c.c_int32, [_c.POINTER(_c.c_char_p), _c.POINTER(_c.c_double),
                                    _c.POINTER(_c.c_double), _c.POINTER(_c.c_int64), _c.c_int32]),
    "tg_directed_row_width": (_c.c_int32, [_c.c_int32]),
    "tg_directed_global_width": (_c.c_int64, [_c.c_int32]),
    "tg_directed_workspace_bytes": (_c.c_size_t, [_c.c_int64, _c.c_int64, _c.c_int32]),
    "tg_count_directed": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                     _c.c_int64, _c.c_int64, _c.c_int32, _c.c_void_p,
                                     _c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "tg_graphlet_weights": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int32, _c.c_void_p,
                                       _c.c_void_p, _c.c_int32, _c.POINTER(_c.c_int32),
                                       _c.c_void_p, _c.c_void_p]),
    "tg_embedding_workspace_bytes": (_c.c_size_t, [_c.c_int64, _c.c_int64, _c.c_int32]),
    "tg_graphlet_embedding": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int64,
                                         _c.c_void_p, _c.c_int32, _c.POINTER(EmbedOpts),
                                         _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                         _c.POINTER(_c.c_int32), _c.c_void_p, _c.c_size_t,
                                         _c.c_void_p]),
}

_lib = None


class TGError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = f"{what}: tg_status {code} ({status_str(code)})"
        if code == 6:
            detail = load().tg_last_error()
            if detail:
                msg += f": {detail.decode()}"
        super().__init__(msg)


def load(path: str | None = None):
    """Load the library (once).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(the typed-graphlet counts only run on the HIP library)")
    # torch's HIP libraries first: they bring the HSA runtime that the
    # library's HIP runtime then shares (loaded the other way round, torch
    # later initialises on the library's HSA runtime and every launch of
    # the library fails with hipErrorNoDevice)
    import torch  # noqa: F401

    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_str(code: int) -> str:
    s = load().tg_status_str(code)
    return s.decode() if s else "?"


def row_width(L: int) -> int:
    return load().tg_row_width(L)


def global_width(L: int) -> int:
    return load().tg_global_width(L)


def workspace_bytes(n: int, nnz: int, L: int) -> int:
    return load().tg_workspace_bytes(n, nnz, L)


def key_describe(L: int, col: int):
    o, t, u = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    rc = load().tg_key_describe(L, col, ctypes.byref(o), ctypes.byref(t), ctypes.byref(u))
    if rc:
        raise TGError(rc, "tg_key_describe")
    return o.value, t.value, u.value


def global_key_describe(L: int, idx: int):
    h, k = ctypes.c_int32(), ctypes.c_int32()
    ts = (ctypes.c_int32 * 4)()
    rc = load().tg_global_key_describe(L, idx, ctypes.byref(h), ts, ctypes.byref(k))
    if rc:
        raise TGError(rc, "tg_global_key_describe")
    return h.value, tuple(ts[: k.value])


def set_timing(enable: bool) -> None:
    load().tg_set_timing(1 if enable else 0)


def phase_times() -> list[tuple[str, float]]:
    ms = (ctypes.c_float * 32)()
    names = (ctypes.c_char_p * 32)()
    cnt = load().tg_phase_times(ms, names, 32)
    return [(names[q].decode(), float(ms[q])) for q in range(max(cnt, 0))]


def kernel_sums() -> dict:
    """Per-class device time of the last directed or embedding call on this
    thread (timing on): {name: {"ms", "units", "calls"}}."""
    k = 32
    names = (ctypes.c_char_p * k)()
    ms = (ctypes.c_double * k)()
    units = (ctypes.c_double * k)()
    calls = (ctypes.c_int64 * k)()
    cnt = load().tg_kernel_sums(names, ms, units, calls, k)
    return {names[q].decode(): {"ms": ms[q], "units": units[q], "calls": int(calls[q])}
            for q in range(cnt)}


TUNE_KNOBS = {"task_wedges": 0, "clear_bytes": 1, "cycle_slots": 2, "map_bytes": 3,
              "edge_slots": 4, "tbuf_bytes": 5, "range_bytes": 6, "derive_edges": 7,
              "light_wedges": 8, "edge_deg": 9, "sh_max": 10, "sh_deg": 11,
              "blk_wedges": 12, "blk_bytes": 13, "blk_task": 14, "blk_wedges_b": 15,
              "hub_lds": 16}


def set_tuning(**knobs) -> dict:
    """Set heavy-path scheduling knobs for this thread; returns the old values."""
    old = {}
    for name, value in knobs.items():
        k = TUNE_KNOBS[name]
        old[name] = load().tg_get_tuning(k)
        rc = load().tg_set_tuning(k, int(value))
        if rc:
            raise TGError(rc, f"tg_set_tuning({name}={value})")
    return old


def get_tuning() -> dict:
    return {name: load().tg_get_tuning(k) for name, k in TUNE_KNOBS.items()}


def last_stats() -> dict:
    st = (ctypes.c_int64 * 14)()
    load().tg_last_stats(st, 14)
    return {"wedges_pass_a": st[0], "light_groups": st[1], "heavy_groups": st[2],
            "heavy_edges": st[3], "wedges_pass_b": st[4], "heavy_wedges_pass_a": st[5],
            "heavy_wedges_pass_b": st[6], "triangle_slots": st[7], "superhub_candidates": st[8],
            "superhubs": st[9], "hub_core": st[10], "blocked_groups": st[11],
            "blocked_wedges_pass_a": st[12], "blocked_wedges_pass_b": st[13]}


def count_raw(row_ptr_ptr: int, col_ptr: int, types_ptr: int, n: int, nnz: int, L: int,
              per_edge_ptr: int, global_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    rc = load().tg_count_typed_graphlets(row_ptr_ptr, col_ptr, types_ptr, n, nnz, L, per_edge_ptr,
                                         global_ptr, ws_ptr, ws_bytes, stream)
    if rc:
        raise TGError(rc, "tg_count_typed_graphlets")


NOALLOC_SCRATCH_BYTES = 256 << 20


def count_noalloc_raw(row_ptr_ptr: int, col_ptr: int, types_ptr: int, n: int, nnz: int, L: int,
                      per_edge_ptr: int, global_ptr: int, stream: int) -> None:
    rc = load().tg_count_typed_graphlets_noalloc(row_ptr_ptr, col_ptr, types_ptr, n, nnz, L,
                                                 per_edge_ptr, global_ptr, stream)
    if rc:
        raise TGError(rc, "tg_count_typed_graphlets_noalloc")


def batch_workspace_bytes(n: int, nnz: int, G: int, L_max: int) -> int:
    return load().tg_batch_workspace_bytes(n, nnz, G, L_max)


def count_batch_raw(row_ptr: int, col: int, types: int, n: int, nnz: int, node_ptr: int,
                    graph_L: int, G: int, L_max: int, goff: int, globals_len: int, per_edge: int,
                    globals_ptr: int, ws: int, ws_bytes: int, stream: int) -> None:
    rc = load().tg_count_batch(row_ptr, col, types, n, nnz, node_ptr, graph_L, G, L_max, goff,
                               globals_len, per_edge, globals_ptr, ws, ws_bytes, stream)
    if rc:
        raise TGError(rc, "tg_count_batch")


def count_batch_async_raw(row_ptr: int, col: int, types: int, n: int, nnz: int, node_ptr: int,
                          graph_L: int, G: int, L_max: int, max_graph_nodes: int, goff: int,
                          globals_len: int, per_edge: int, globals_ptr: int, ws: int,
                          ws_bytes: int, status_out: int, stream: int) -> None:
    rc = load().tg_count_batch_async(row_ptr, col, types, n, nnz, node_ptr, graph_L, G, L_max,
                                     max_graph_nodes, goff, globals_len, per_edge, globals_ptr, ws,
                                     ws_bytes, status_out, stream)
    if rc:
        raise TGError(rc, "tg_count_batch_async")


def sparse_workspace_bytes(m: int) -> int:
    return int(load().tg_sparse_workspace_bytes(m))


def sparse_offsets_raw(rows_ptr: int, m: int, L: int, off_ptr: int, ws_ptr: int, ws_bytes: int,
                       stream: int) -> None:
    rc = load().tg_sparse_offsets(rows_ptr, m, L, off_ptr, ws_ptr, ws_bytes, stream)
    if rc:
        raise TGError(rc, "tg_sparse_offsets")


def sparse_fill_raw(rows_ptr: int, m: int, L: int, off_ptr: int, keys_ptr: int, counts_ptr: int,
                    stream: int) -> None:
    rc = load().tg_sparse_fill(rows_ptr, m, L, off_ptr, keys_ptr, counts_ptr, stream)
    if rc:
        raise TGError(rc, "tg_sparse_fill")


# ------------------------------------------------ position-aware (Sec. 5)

PA_BLOCKS = ["tri", "path_i", "path_j", "g3i", "g3j", "g4", "g5i", "g5j", "g6", "g7i", "g7j",
             "g8", "g9i", "g9j", "g10i", "g10j", "g11", "g12"]


def pa_row_width(L: int) -> int:
    return load().tg_pa_row_width(L)


def pa_global_width(L: int) -> int:
    return int(load().tg_pa_global_width(L))


def pa_key_describe(L: int, col: int):
    """(block name, t, t2) of position-aware column col."""
    b, t, u = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    rc = load().tg_pa_key_describe(L, col, ctypes.byref(b), ctypes.byref(t), ctypes.byref(u))
    if rc:
        raise TGError(rc, "tg_pa_key_describe")
    return PA_BLOCKS[b.value], t.value, u.value


def pa_global_key_describe(L: int, idx: int):
    """(graphlet 0..8, types by drawing position) of global class idx."""
    h, k = ctypes.c_int32(), ctypes.c_int32()
    ts = (ctypes.c_int32 * 4)()
    rc = load().tg_pa_global_key_describe(L, idx, ctypes.byref(h), ts, ctypes.byref(k))
    if rc:
        raise TGError(rc, "tg_pa_global_key_describe")
    return h.value, tuple(ts[: k.value])


def count_position_aware_raw(row_ptr: int, col: int, types: int, n: int, nnz: int, L: int,
                             per_edge: int, glob: int, ws: int, ws_bytes: int,
                             stream: int) -> None:
    rc = load().tg_count_position_aware(row_ptr, col, types, n, nnz, L, per_edge, glob, ws,
                                        ws_bytes, stream)
    if rc:
        raise TGError(rc, "tg_count_position_aware")
