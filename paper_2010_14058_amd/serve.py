"""Serving driver over the library's native server (``tg_server_*`` in
``include/tg.h``): admission by HBM footprint, device-resident CSR and
results, continuous batching on several workers with their own streams,
all inside ``libtg.so``.  This module only allocates the device arena (a
torch tensor), submits requests from host arrays, collects each finished
request's global vector and releases it, and reports latencies from the
server's own timestamps.
"""

from __future__ import annotations

import ctypes
import dataclasses
import threading
import time

import numpy as np

from . import _lib

TG_E_OOM = 10


@dataclasses.dataclass
class Request:
    rid: int
    row_ptr: np.ndarray      # int64 [n+1]
    col: np.ndarray          # int32 [nnz]
    types: np.ndarray        # uint8 [n]
    L: int
    arrival: float = 0.0     # seconds after the replay's start
    status: int = -1         # tg_status once finished (0 = ok), -1 while pending
    error: str = ""
    result: np.ndarray | None = None   # uint64 global counts (own L layout)
    ticket: int = -1
    batch: int = -1
    t_submit: float = -1.0   # server clock (seconds since its creation)
    t_admit: float = -1.0
    t_start: float = -1.0
    t_done: float = -1.0

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col.shape[0] // 2)


class Server:
    """A native server on a device arena of ``hbm_budget`` bytes."""

    def __init__(self, hbm_budget: int, workers: int = 2, worker_bytes: int | None = None,
                 single_edges: int = 1 << 17, max_batch_edges: int = 8_000_000, device=None):
        import torch

        self.budget = int(hbm_budget)
        self.workers = int(workers)
        if worker_bytes is None:
            worker_bytes = (self.budget * 3 // 4) // self.workers
        self.worker_bytes = int(worker_bytes) & ~255
        self.arena = torch.empty(self.budget, dtype=torch.uint8, device=device or "cuda")
        self.handle = ctypes.c_void_p()
        rc = _lib.load().tg_server_create(self.arena.data_ptr(), self.budget, self.workers,
                                          self.worker_bytes, int(single_edges),
                                          int(max_batch_edges), ctypes.byref(self.handle))
        if rc:
            raise _lib.TGError(rc, "tg_server_create")
        self.lock = threading.Lock()
        self.pending: dict[int, Request] = {}
        self.done: list[Request] = []
        self.rejected = 0
        self.closed = False
        self.t_first = None
        self.collector = threading.Thread(target=self._collect, daemon=True)
        self.collector.start()

    def submit(self, req: Request) -> None:
        lib = _lib.load()
        rp = np.ascontiguousarray(req.row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(req.col, dtype=np.int32)
        ty = np.ascontiguousarray(req.types, dtype=np.uint8)
        desc = _lib.GraphDesc(rp.ctypes.data, col.ctypes.data if col.size else 0, ty.ctypes.data,
                              req.n, int(col.size), int(req.L), 0)
        ticket = ctypes.c_int64(-1)
        with self.lock:  # registered before the collector can see it finish
            rc = lib.tg_server_submit(self.handle, ctypes.byref(desc), ctypes.byref(ticket))
            if rc:
                req.status = rc
                req.error = _lib.status_str(rc)
                self.rejected += int(rc == TG_E_OOM)
                self.done.append(req)
                return
            req.ticket = int(ticket.value)
            self.pending[req.ticket] = req

    def _finish(self, req: Request) -> None:
        lib = _lib.load()
        info = _lib.RequestInfo()
        if lib.tg_server_poll(self.handle, req.ticket, ctypes.byref(info)):
            return
        req.status = int(info.status)
        req.t_submit, req.t_admit = info.t_submit, info.t_admit
        req.t_start, req.t_done, req.batch = info.t_start, info.t_done, int(info.batch)
        if req.status == 0 and info.global_counts:
            off = int(info.global_counts) - self.arena.data_ptr()
            w = _lib.global_width(req.L)
            req.result = self.arena[off:off + 8 * w].cpu().numpy().view(np.uint64).copy()
        elif req.status:
            req.error = _lib.status_str(req.status)
        lib.tg_server_release(self.handle, req.ticket)

    def _collect(self) -> None:
        lib = _lib.load()
        buf = (ctypes.c_int64 * 4096)()
        while True:
            with self.lock:
                if not self.pending and self.closed:
                    return
            k = lib.tg_server_take_done(self.handle, buf, 4096, 0.005)
            for q in range(k):
                with self.lock:
                    req = self.pending.pop(int(buf[q]), None)
                if req is None:
                    continue
                self._finish(req)
                with self.lock:
                    self.done.append(req)

    def close(self, timeout: float | None = None) -> None:
        """Wait until every submitted request has finished, then stop."""
        t_end = None if timeout is None else time.perf_counter() + timeout
        while True:
            with self.lock:
                if not self.pending:
                    break
            if t_end is not None and time.perf_counter() > t_end:
                raise TimeoutError("requests still pending")
            time.sleep(0.001)
        with self.lock:
            self.closed = True
        self.collector.join()
        self.stats = self.server_stats()
        rc = _lib.load().tg_server_destroy(self.handle)
        self.arena = None            # results were copied out; the device memory goes back
        if rc:
            raise _lib.TGError(rc, "tg_server_destroy")

    def server_stats(self) -> dict:
        st = (ctypes.c_int64 * 12)()
        _lib.load().tg_server_stats(self.handle, st, 12)
        names = ["submitted", "finished", "rejected", "batches", "single_calls", "pool_in_use",
                 "peak_pool_bytes", "pool_bytes", "busy_us", "waiting", "admitted", "device_error"]
        return dict(zip(names, (int(x) for x in st)))

    def report(self) -> dict:
        ok = [r for r in self.done if r.status == 0]
        lat = np.array([r.t_done - r.t_submit for r in ok]) if ok else np.zeros(1)
        t_first = min((r.t_submit for r in ok), default=0.0)
        t_last = max((r.t_done for r in ok), default=1e-9)
        span = max(t_last - t_first, 1e-9)
        edges = sum(r.m for r in ok)
        st = getattr(self, "stats", None) or self.server_stats()
        return {
            "requests": len(self.done),
            "ok": len(ok),
            "rejected": self.rejected + int(st.get("rejected", 0)),
            "batches": st.get("batches"),
            "single_calls": st.get("single_calls"),
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "served_edges_per_s": edges / span,
            "served_graphs_per_s": len(ok) / span,
            "span_s": span,
            "worker_busy_fraction": st.get("busy_us", 0) * 1e-6 / (span * self.workers),
            "peak_pool_bytes": st.get("peak_pool_bytes"),
            "pool_bytes": st.get("pool_bytes"),
            "worker_bytes": self.worker_bytes,
        }


def replay(srv: Server, reqs: list[Request], clock=time.perf_counter) -> None:
    """Submit each request at its arrival time (relative to now)."""
    t0 = clock()
    for r in sorted(reqs, key=lambda r: r.arrival):
        delay = r.arrival - (clock() - t0)
        if delay > 0:
            time.sleep(delay)
        srv.submit(r)
