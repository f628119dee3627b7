"""C ABI checks that need no GPU: the library loads, exports every function
the header declares, and its layout helpers agree with the documented
layout (checked against the brute-force module's own enumeration)."""

import ctypes
import os
import re

import pytest

import brute_force as BF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tg.h")


def _lib():
    from paper_2010_14058_amd import _lib as L

    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libtg.so not built")
    return L


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(tg_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_symbols_exported():
    L = _lib()
    lib = ctypes.CDLL(L.LIB_PATH)
    names = header_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    # the binding declares exactly the header's functions
    assert sorted(L.SIGNATURES) == names


def test_widths_and_workspace():
    L = _lib()
    for nt in range(1, 17):
        assert L.row_width(nt) == 2 * nt + 10 * (nt * (nt + 1) // 2)
        assert L.global_width(nt) == len(BF.multisets(nt, 2)) + 2 * len(BF.multisets(nt, 3)) + 6 * len(
            BF.multisets(nt, 4))
    assert L.row_width(0) == 0 and L.row_width(17) == 0
    assert L.workspace_bytes(1000, 8000, 3) > 0
    assert L.workspace_bytes(1000, 8001, 3) == 0      # odd nnz
    assert L.workspace_bytes(10, 20, 0) == 0          # L out of range


@pytest.mark.parametrize("nt", [1, 3, 5, 8])
def test_key_describe(nt):
    L = _lib()
    idx = BF.column_index(nt)
    for name, c in idx.items():
        o, t, u = L.key_describe(nt, c)
        if name.startswith("tri"):
            assert (o, u) == (1, -1) and name == f"tri[{t}]"
        elif name.startswith("path3"):
            assert (o, u) == (2, -1) and name == f"path3[{t}]"
        else:
            assert name == f"g{o}[{t},{u}]"


@pytest.mark.parametrize("nt", [1, 2, 4, 6])
def test_global_key_describe(nt):
    L = _lib()
    q = 0
    for h, k in [(0, 2), (1, 3), (2, 3)] + [(h, 4) for h in range(3, 9)]:
        for ms in BF.multisets(nt, k):
            assert L.global_key_describe(nt, q) == (h, ms)
            q += 1
    assert q == L.global_width(nt)


def test_tuning_knobs():
    import paper_2010_14058_amd as P

    base = P.get_tuning()
    assert base["task_wedges"] == 1 << 18 and base["clear_bytes"] == 64
    assert base["cycle_slots"] >= 1 and base["edge_slots"] >= 1
    old = P.set_tuning(task_wedges=100, clear_bytes=0)
    assert old == {"task_wedges": 1 << 18, "clear_bytes": 64}
    now = P.get_tuning()
    assert now["task_wedges"] == 100 and now["clear_bytes"] == 0
    ws = P.workspace_bytes(1000, 8000, 5)
    P.set_tuning(cycle_slots=1)
    assert 0 < P.workspace_bytes(1000, 8000, 5) < ws
    with pytest.raises(P.TGError):
        P.set_tuning(edge_slots=0)
    with pytest.raises(P.TGError):
        P.set_tuning(task_wedges=0)
    with pytest.raises(P.TGError):
        P.set_tuning(clear_bytes=-1)
    # degree buckets: defaults are the largest buckets the kernels support
    assert base["light_wedges"] == 512 and base["edge_deg"] == 1024
    P.set_tuning(light_wedges=1, edge_deg=1)
    for bad in ({"light_wedges": 0}, {"light_wedges": 513}, {"edge_deg": 0}, {"edge_deg": 1025}):
        with pytest.raises(P.TGError):
            P.set_tuning(**bad)
    # blocked 4-cycle path: its record space is workspace, 0 turns it off
    assert base["blk_wedges"] == 1 << 16 and base["blk_bytes"] == 4 << 30
    assert base["blk_task"] == 1 << 16 and base["blk_wedges_b"] == 1 << 31
    assert base["hub_lds"] == 20480
    # (a graph of 8e5 adjacency slots may need the whole 4 GiB of records;
    # a small one gets at most nnz^2 / 2 records)
    with_blk = P.workspace_bytes(100000, 800000, 5)
    small_blk = P.workspace_bytes(1000, 8000, 5)
    P.set_tuning(blk_bytes=0)
    assert 0 < P.workspace_bytes(100000, 800000, 5) < with_blk - (4 << 30) + (1 << 20)
    assert 0 < P.workspace_bytes(1000, 8000, 5) < small_blk <= \
        P.workspace_bytes(1000, 8000, 5) + 8000 * 8000 + (4 << 20)
    for bad in ({"blk_wedges": 0}, {"blk_bytes": -1}, {"blk_bytes": (8 << 30) + 1},
                {"blk_task": 1023}, {"blk_task": (1 << 16) + 1}, {"blk_wedges_b": 0},
                {"hub_lds": -1}, {"hub_lds": 65537}):
        with pytest.raises(P.TGError):
            P.set_tuning(**bad)
    P.set_tuning(**base)
    assert P.get_tuning() == base


def test_sparse_argument_checks():
    """Argument checks of the sparse-output calls happen before any device work."""
    from paper_2010_14058_amd import _lib as L

    lib = L.load()
    assert L.sparse_workspace_bytes(10) > 0
    assert lib.tg_sparse_workspace_bytes(-1) == 0
    assert lib.tg_sparse_offsets(None, 4, 0, None, None, 0, None) == 4   # TG_E_L_RANGE
    assert lib.tg_sparse_offsets(None, -1, 3, 1, 1, 0, None) == 1        # negative m
    assert lib.tg_sparse_offsets(None, 4, 3, 1, 1, 1 << 40, None) == 1   # rows missing
    assert lib.tg_sparse_offsets(1, 4, 3, 1, 1, 0, None) == 5            # workspace too small
    assert lib.tg_sparse_fill(None, 4, 17, 1, 1, 1, None) == 4
    assert lib.tg_sparse_fill(1, 4, 3, 1, None, 1, None) == 1
    assert lib.tg_sparse_fill(None, 0, 3, 1, None, None, None) == 0      # nothing to do


def test_workspace_alignment_checked_first():
    """A workspace that is not 256-byte aligned is refused before any device
    work (the pointers are never dereferenced)."""
    from paper_2010_14058_amd import _lib as L

    lib = L.load()
    n, nnz, nt = 100, 400, 3
    need = lib.tg_workspace_bytes(n, nnz, nt)
    assert need > 0
    fake = 1 << 20
    assert lib.tg_count_typed_graphlets(fake, fake, fake, n, nnz, nt, None, None,
                                        fake + 16, need, None) == 1   # TG_E_INVALID_ARG
    assert lib.tg_count_typed_graphlets(fake, fake, fake, n, nnz, nt, None, None,
                                        fake, need - 1, None) == 5    # TG_E_WORKSPACE
    G = 2
    bneed = lib.tg_batch_workspace_bytes(n, nnz, G, nt)
    assert bneed > 0
    assert lib.tg_count_batch(fake, fake, fake, n, nnz, fake, fake, G, nt, fake, 10, None, fake,
                              fake + 64, bneed, None) == 1


def test_noalloc_rejects_oversized_graph():
    """A graph whose workspace exceeds the static scratch is refused before
    any device work (no GPU needed to see it)."""
    L = _lib()
    lib = L.load()
    dummy = ctypes.c_void_p(8)  # never dereferenced: the size check comes first
    rc = lib.tg_count_typed_graphlets_noalloc(dummy, dummy, dummy, 50_000_000, 0, 5, None, None,
                                              None)
    assert rc == 8  # TG_E_TOO_LARGE
    assert lib.tg_count_typed_graphlets_noalloc(dummy, dummy, dummy, 10, 3, 5, None, None,
                                                None) == 1  # odd nnz
    assert lib.tg_count_typed_graphlets_noalloc(dummy, dummy, dummy, 10, 2, 0, None, None,
                                                None) == 4  # L out of range


@pytest.mark.parametrize("nt", [1, 2, 3, 5])
def test_pa_layout_matches_oracle(oracle_mod, nt):
    """The library's position-aware row and global layouts (closed-form
    ranks) agree with the oracle's (tables built by enumeration): column by
    column, and class by class up to type-preserving isomorphism."""
    L = _lib()
    assert L.pa_row_width(nt) == oracle_mod.pa_row_width(nt) == 3 * nt + 9 * nt * nt + 6 * (
        nt * (nt + 1) // 2)
    W = L.pa_global_width(nt)
    assert W == oracle_mod.pa_global_width(nt)
    for c, name in enumerate(oracle_mod.pa_column_names(nt)):
        b, t, u = L.pa_key_describe(nt, c)
        if u < 0:
            mine = f"{b}[{t}]"
        elif b in BF.PA_PAIR:
            mine = f"{b}{{{t},{u}}}"
        else:
            mine = f"{b}[{t},{u}]"
        assert mine == name
    for idx in range(W):
        h, lab = L.pa_global_key_describe(nt, idx)
        h2, lab2 = oracle_mod.pa_global_describe(nt, idx)
        assert h == h2
        assert BF.pa_class_key(h, lab, nt) == BF.pa_class_key(h2, lab2, nt), (idx, lab, lab2)


def test_pa_widths_all_L():
    import math

    L = _lib()
    for nt in range(1, 17):
        P = nt * (nt + 1) // 2
        classes = [P, nt * P, math.comb(nt + 2, 3), (nt ** 4 + nt ** 2) // 2,
                   nt * math.comb(nt + 2, 3), (nt ** 4 + 2 * nt ** 3 + 3 * nt ** 2 + 2 * nt) // 8,
                   nt * nt * P, P * P, math.comb(nt + 3, 4)]
        assert L.pa_global_width(nt) == sum(classes)
        assert L.pa_row_width(nt) == 3 * nt + 9 * nt * nt + 6 * P
    assert L.pa_row_width(0) == 0 and L.pa_global_width(17) == 0


def test_embedding_argument_checks():
    """Argument errors of the embedding calls, all caught before any device
    work."""
    import ctypes

    import paper_2010_14058_amd as P

    lib = P._lib.load()
    ms = (ctypes.c_int32 * 4)(0, 0, 0, 0)
    assert lib.tg_graphlet_weights(None, 0, 0, None, None, 0, ms, None, None) == 4  # L range
    assert lib.tg_graphlet_weights(None, 0, 2, None, None, 9, ms, None, None) == 1  # graphlet
    assert lib.tg_graphlet_weights(None, -1, 2, None, None, 0, ms, None, None) == 1
    bad = (ctypes.c_int32 * 4)(1, 0, 0, 0)
    assert lib.tg_graphlet_weights(None, 0, 2, None, None, 0, bad, None, None) == 3  # unsorted
    big = (ctypes.c_int32 * 4)(0, 2, 0, 0)
    assert lib.tg_graphlet_weights(None, 0, 2, None, None, 0, big, None, None) == 3  # type >= L
    assert lib.tg_graphlet_weights(None, 0, 2, None, None, 2, ms, None, None) == 0  # m = 0
    assert lib.tg_embedding_workspace_bytes(10, 20, 0) == 0
    assert lib.tg_embedding_workspace_bytes(10, 20, 257) == 0
    ws = lib.tg_embedding_workspace_bytes(1000, 8000, 16)
    assert ws > 1000 * 24 * 8 * 5
    opts = P._lib.EmbedOpts(0, 0, 0.0, 0, 0, 0)
    its = ctypes.c_int32(0)
    fake = 1 << 20  # never dereferenced: every call below fails its checks first
    call = lambda n, nnz, dim, wsp, wsb: lib.tg_graphlet_embedding(
        fake, fake, n, nnz, fake, dim, ctypes.byref(opts), fake, None, None, ctypes.byref(its),
        wsp, wsb, None)
    assert call(1000, 8000, 0, fake, ws) == 1      # dim
    assert call(1000, 8000, 257, fake, ws) == 1
    assert call(1000, 8001, 16, fake, ws) == 1     # odd nnz
    assert call(0, 0, 16, fake, ws) == 1           # n < 1
    assert call(1000, 8000, 16, fake + 8, ws) == 1  # unaligned workspace
    assert call(1000, 8000, 16, fake, ws - 1) == 5  # workspace too small
    assert call(1 << 31, 8000, 16, fake, ws) == 8   # too large
