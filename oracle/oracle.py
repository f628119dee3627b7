"""ctypes front end of the C oracle in ``tg_oracle.c``.

``build_oracle()`` compiles it with gcc into ``oracle/liboracle.so``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_ERRS = {1: "invalid argument", 2: "out of memory", 3: "global count not divisible by |E(H)|",
         4: "negative derived count"}


def build_oracle(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle()
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.tgo_row_width.argtypes = [ctypes.c_int]
        lib.tgo_global_width.argtypes = [ctypes.c_int]
        lib.tgo_pair_index.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.tgo_edge_definition.argtypes = [i64, p, p, p, ctypes.c_int, i32, i32, p]
        lib.tgo_edge_paper.argtypes = [i64, p, p, p, ctypes.c_int, i32, i32, p]
        lib.tgo_edges.argtypes = [i64, p, p, p, ctypes.c_int, p, i64, ctypes.c_int,
                                  ctypes.c_int, p]
        lib.tgo_global_from_rows.argtypes = [p, ctypes.c_int, p, i64, p, p]
        lib.tgo_pa_row_width.argtypes = [ctypes.c_int]
        lib.tgo_pa_global_width.argtypes = [ctypes.c_int]
        lib.tgo_pa_global_width.restype = i64
        lib.tgo_pa_edges.argtypes = [i64, p, p, p, ctypes.c_int, p, i64, ctypes.c_int,
                                     ctypes.c_int, p]
        lib.tgo_pa_global_from_rows.argtypes = [p, ctypes.c_int, p, i64, p, p]
        lib.tgo_pa_global_describe.argtypes = [ctypes.c_int, i64, p, p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _check(rc: int):
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}: {_ERRS.get(rc, 'unknown')}")


def row_width(L: int) -> int:
    return _load().tgo_row_width(L)


def global_width(L: int) -> int:
    return _load().tgo_global_width(L)


def pair_index(L: int, t: int, u: int) -> int:
    return _load().tgo_pair_index(L, t, u)


def column_names(L: int) -> list[str]:
    names = [f"tri[{t}]" for t in range(L)] + [f"path3[{t}]" for t in range(L)]
    for g in range(3, 13):
        names += [f"g{g}[{t},{u}]" for t in range(L) for u in range(t, L)]
    return names


def _arrays(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    ty = np.ascontiguousarray(g.types, dtype=np.uint8)
    return rp, col, ty


def edge_row(g, i: int, j: int, method: str = "paper") -> np.ndarray:
    """Row of one edge (i, j) in the orientation given."""
    rp, col, ty = _arrays(g)
    out = np.zeros(row_width(g.L), dtype=np.uint64)
    fn = _load().tgo_edge_paper if method == "paper" else _load().tgo_edge_definition
    _check(fn(g.n, _ptr(rp), _ptr(col), _ptr(ty), g.L, int(i), int(j), _ptr(out)))
    return out


def edge_rows(g, uv: np.ndarray, method: str = "paper", threads: int | None = None) -> np.ndarray:
    """Rows for edges uv[k, 2] (each (i, j) in the orientation given)."""
    rp, col, ty = _arrays(g)
    uv = np.ascontiguousarray(uv, dtype=np.int64).reshape(-1, 2)
    out = np.zeros((uv.shape[0], row_width(g.L)), dtype=np.uint64)
    if uv.shape[0] == 0:
        return out
    threads = threads or os.cpu_count() or 1
    m = 1 if method == "paper" else 0
    _check(_load().tgo_edges(g.n, _ptr(rp), _ptr(col), _ptr(ty), g.L, _ptr(uv),
                             uv.shape[0], m, int(threads), _ptr(out)))
    return out


def all_edge_rows(g, method: str = "paper", threads: int | None = None) -> np.ndarray:
    """Rows of every edge (u < v) in lexicographic order."""
    return edge_rows(g, g.edges(), method=method, threads=threads)


def global_counts(g, rows: np.ndarray) -> np.ndarray:
    """Global typed graphlet counts from the rows of all edges (lexicographic)."""
    uv = np.ascontiguousarray(g.edges(), dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    ty = np.ascontiguousarray(g.types, dtype=np.uint8)
    out = np.zeros(global_width(g.L), dtype=np.uint64)
    _check(_load().tgo_global_from_rows(_ptr(ty), g.L, _ptr(uv), uv.shape[0], _ptr(rows),
                                        _ptr(out)))
    return out


# ------------------------------------------------ position-aware (Sec. 5)

PA_BLOCKS = ["tri", "path_i", "path_j", "g3i", "g3j", "g4", "g5i", "g5j", "g6", "g7i", "g7j",
             "g8", "g9i", "g9j", "g10i", "g10j", "g11", "g12"]
PA_PAIR_BLOCKS = {"g5i", "g5j", "g7i", "g7j", "g11", "g12"}


def pa_row_width(L: int) -> int:
    return _load().tgo_pa_row_width(L)


def pa_global_width(L: int) -> int:
    return int(_load().tgo_pa_global_width(L))


def pa_column_names(L: int) -> list[str]:
    """Names of the position-aware row's columns: block[x,y] for ordered
    role pairs, block{t,u} for unordered ones, block[t] for 3-node blocks."""
    names = []
    for b in PA_BLOCKS:
        if b in ("tri", "path_i", "path_j"):
            names += [f"{b}[{t}]" for t in range(L)]
        elif b in PA_PAIR_BLOCKS:
            names += [f"{b}{{{t},{u}}}" for t in range(L) for u in range(t, L)]
        else:
            names += [f"{b}[{x},{y}]" for x in range(L) for y in range(L)]
    return names


def pa_edge_rows(g, uv: np.ndarray, method: str = "paper", threads: int | None = None) -> np.ndarray:
    """Position-aware rows for edges uv[k, 2], each oriented as given."""
    rp, col, ty = _arrays(g)
    uv = np.ascontiguousarray(uv, dtype=np.int64).reshape(-1, 2)
    out = np.zeros((uv.shape[0], pa_row_width(g.L)), dtype=np.uint64)
    if uv.shape[0] == 0:
        return out
    threads = threads or os.cpu_count() or 1
    m = 1 if method == "paper" else 0
    _check(_load().tgo_pa_edges(g.n, _ptr(rp), _ptr(col), _ptr(ty), g.L, _ptr(uv),
                                uv.shape[0], m, int(threads), _ptr(out)))
    return out


def pa_all_edge_rows(g, method: str = "paper", threads: int | None = None) -> np.ndarray:
    """Position-aware rows of every edge (u < v, oriented u -> v), lexicographic."""
    return pa_edge_rows(g, g.edges(), method=method, threads=threads)


def pa_global_counts(g, rows: np.ndarray) -> np.ndarray:
    """Global position-aware counts (classes under type-preserving
    isomorphism) from the position-aware rows of all edges."""
    uv = np.ascontiguousarray(g.edges(), dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    ty = np.ascontiguousarray(g.types, dtype=np.uint8)
    out = np.zeros(pa_global_width(g.L), dtype=np.uint64)
    _check(_load().tgo_pa_global_from_rows(_ptr(ty), g.L, _ptr(uv), uv.shape[0], _ptr(rows),
                                           _ptr(out)))
    return out


def pa_global_describe(L: int, idx: int):
    """(graphlet 0..8, types by node position) of global class idx."""
    h = ctypes.c_int()
    ts = (ctypes.c_int * 4)()
    k = _load().tgo_pa_global_describe(L, idx, ctypes.byref(h), ts)
    if k == 0:
        raise IndexError(idx)
    return h.value, tuple(ts[:k])
