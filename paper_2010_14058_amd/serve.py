"""Serving loop: continuous batching of typed-graphlet count requests.

Requests carry one typed graph each and arrive over time.  The server

* admits a request when its HBM footprint fits the remaining budget
  (footprint = its CSR on the device + the workspace and outputs its own
  call would need, an upper bound of its share of a batched call); a request
  larger than the whole budget is rejected;
* uploads an admitted request's CSR to the device, where it stays until the
  request completes;
* runs several workers, each with its own HIP stream and workspace; a free
  worker takes every admitted request not yet started as one batch (up to
  an edge budget), so requests that arrive while others are on the GPU join
  the next batch and batches of different workers overlap on the device;
* runs the small requests of a batch through one ``tg_count_batch`` call and
  each large one (at least ``single_edges`` edges) through its own
  single-graph call, which keeps the hub core and super-hub bitmaps that a
  batch's graph-major order gives up; every request gets its own global
  count vector; if a batch fails, its requests are re-run one by one so only
  the offending request gets the error.

The executor (batch of requests -> per-request results) is injectable; the
default one calls the HIP library.
"""

from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    row_ptr: np.ndarray      # int64 [n+1]
    col: np.ndarray          # int32 [nnz]
    types: np.ndarray        # uint8 [n]
    L: int
    arrival: float = 0.0     # seconds after the server's start
    status: int = -1         # tg_status once finished (0 = ok), -1 while pending
    error: str = ""
    result: np.ndarray | None = None   # uint64 global counts (own L layout)
    t_admit: float = -1.0
    t_start: float = -1.0
    t_done: float = -1.0
    footprint: int = 0
    device: dict | None = None         # device-resident CSR while admitted

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col.shape[0] // 2)


TG_E_OOM = 100  # status of a request whose footprint exceeds the whole budget


def footprint_bytes(n: int, nnz: int, L: int) -> int:
    """HBM a request may occupy: CSR, types, its own workspace and outputs."""
    from . import _lib

    ws = _lib.workspace_bytes(max(n, 1), nnz, L)
    return 8 * (n + 1) + 4 * nnz + n + ws + 8 * _lib.global_width(L)


class Server:
    def __init__(self, hbm_budget: int, executor: Callable | None = None, workers: int = 2,
                 max_batch_edges: int = 8_000_000, footprint: Callable | None = None,
                 uploader: Callable | None = None, clock: Callable = time.perf_counter):
        self.budget = int(hbm_budget)
        self.in_use = 0
        self.executor = executor or GpuExecutor()
        self.footprint = footprint or (lambda r: footprint_bytes(r.n, 2 * r.m, r.L))
        self.uploader = uploader or getattr(self.executor, "upload", None)
        self.max_batch_edges = int(max_batch_edges)
        self.clock = clock
        self.t0 = clock()
        self.lock = threading.Condition()
        self.waiting = collections.deque()   # arrived, not admitted
        self.ready = collections.deque()     # admitted (on device), not started
        self.done: list[Request] = []
        self.rejected = 0
        self.batches = 0
        self.batch_sizes: list[int] = []
        self.closed = False
        self.workers = [threading.Thread(target=self._worker, args=(w,), daemon=True)
                        for w in range(workers)]
        for t in self.workers:
            t.start()

    # ------------------------------------------------------------ public
    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request) -> None:
        req.footprint = int(self.footprint(req))
        with self.lock:
            if req.footprint > self.budget:
                req.status = TG_E_OOM
                req.error = "request larger than the HBM budget"
                req.t_done = self.now()
                self.rejected += 1
                self.done.append(req)
                self.lock.notify_all()
                return
            self.waiting.append(req)
            self._admit_locked()
            self.lock.notify_all()

    def close(self, timeout: float | None = None) -> None:
        """Wait until every submitted request has finished, then stop."""
        with self.lock:
            self.lock.wait_for(lambda: not self.waiting and not self.ready and
                               self._running == 0, timeout=timeout)
            self.closed = True
            self.lock.notify_all()
        for t in self.workers:
            t.join(timeout=timeout)

    # ---------------------------------------------------------- internals
    _running = 0

    def _admit_locked(self) -> None:
        # FIFO admission: the head waits until it fits (no overtaking)
        while self.waiting and self.in_use + self.waiting[0].footprint <= self.budget:
            r = self.waiting.popleft()
            self.in_use += r.footprint
            r.t_admit = self.now()
            if self.uploader is not None:
                r.device = self.uploader(r)
            self.ready.append(r)

    def _take_batch_locked(self) -> list[Request]:
        batch, edges = [], 0
        while self.ready and (not batch or edges + self.ready[0].m <= self.max_batch_edges):
            r = self.ready.popleft()
            edges += r.m
            batch.append(r)
        return batch

    def _worker(self, w: int) -> None:
        while True:
            with self.lock:
                self.lock.wait_for(lambda: self.ready or self.closed)
                if not self.ready and self.closed:
                    return
                batch = self._take_batch_locked()
                self._running += 1
                self.batches += 1
                self.batch_sizes.append(len(batch))
            t = self.now()
            for r in batch:
                r.t_start = t
            try:
                results = self.executor.run(batch, w)
                statuses = [(0, "")] * len(batch)
            except Exception as exc:  # isolate the failing request(s)
                results, statuses = [], []
                for r in batch:
                    try:
                        results.append(self.executor.run([r], w)[0])
                        statuses.append((0, ""))
                    except Exception as exc1:
                        results.append(None)
                        statuses.append((getattr(exc1, "code", 7), str(exc1)))
                del exc
            t = self.now()
            with self.lock:
                for r, res, (st, msg) in zip(batch, results, statuses):
                    r.result = res
                    r.status = st
                    r.error = msg
                    r.t_done = t
                    r.device = None
                    self.in_use -= r.footprint
                    self.done.append(r)
                self._running -= 1
                self._admit_locked()
                self.lock.notify_all()

    # ------------------------------------------------------------- report
    def report(self) -> dict:
        ok = [r for r in self.done if r.status == 0]
        lat = np.array([r.t_done - r.arrival for r in ok]) if ok else np.zeros(1)
        first = min((r.arrival for r in self.done), default=0.0)
        last = max((r.t_done for r in self.done), default=0.0)
        span = max(last - first, 1e-9)
        edges = sum(r.m for r in ok)
        return {
            "requests": len(self.done), "completed": len(ok), "rejected": self.rejected,
            "failed": len(self.done) - len(ok) - self.rejected,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "served_edges_per_s": edges / span, "served_graphs_per_s": len(ok) / span,
            "batches": self.batches,
            "mean_batch_graphs": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
        }


class GpuExecutor:
    """Runs a batch of requests on one HIP device.

    Worker w uses its own stream and workspace.  A request's CSR is uploaded
    at admission.  Requests of fewer than ``single_edges`` edges are
    concatenated on the device into one union CSR and counted by one
    ``tg_count_batch`` call; larger ones are counted one
    ``tg_count_typed_graphlets`` call each (global counts only), on the same
    stream.
    """

    def __init__(self, device: str = "cuda:0", workers: int = 2, single_edges: int = 1 << 17):
        import torch

        from . import Workspace

        self.single_edges = int(single_edges)
        self.dev = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(workers)]
        self.ws = [Workspace(self.dev) for _ in range(workers)]
        self.upload_stream = torch.cuda.Stream(device=self.dev)

    def upload(self, r: Request) -> dict:
        import torch

        with torch.cuda.stream(self.upload_stream):
            d = {
                "row_ptr": torch.from_numpy(r.row_ptr).pin_memory().to(self.dev, non_blocking=True),
                "col": torch.from_numpy(r.col).pin_memory().to(self.dev, non_blocking=True),
                "types": torch.from_numpy(r.types).pin_memory().to(self.dev, non_blocking=True),
            }
            ev = torch.cuda.Event()
            ev.record(self.upload_stream)
        d["ready"] = ev
        return d

    def run(self, batch: list[Request], w: int) -> list[np.ndarray]:
        import torch

        from . import count_typed_graphlets

        stream = self.streams[w % len(self.streams)]
        ws = self.ws[w % len(self.ws)]
        out: list = [None] * len(batch)
        with torch.cuda.stream(stream):
            for r in batch:
                if r.device is None:
                    r.device = self.upload(r)
                stream.wait_event(r.device["ready"])
            small = [q for q, r in enumerate(batch) if r.m < self.single_edges]
            if small:
                for q, res in zip(small, self._run_batched([batch[q] for q in small], ws, stream)):
                    out[q] = res
            for q, r in enumerate(batch):
                if r.m < self.single_edges:
                    continue
                d = r.device
                _, g1 = count_typed_graphlets(d["row_ptr"], d["col"], d["types"], r.L,
                                              per_edge=False, workspace=ws, stream=stream)
                out[q] = g1.cpu().numpy().view(np.uint64).copy()
        return out

    def _run_batched(self, batch: list[Request], ws, stream) -> list[np.ndarray]:
        """One tg_count_batch call over the union of the requests' graphs
        (on the current stream, which is ``stream``)."""
        import torch

        from . import BatchPlan, count_batch

        nodes = np.array([0] + [r.n for r in batch], dtype=np.int64)
        node_off = np.cumsum(nodes)
        nnz = np.array([0] + [2 * r.m for r in batch], dtype=np.int64)
        nnz_off = np.cumsum(nnz)
        row_parts = [torch.zeros(1, dtype=torch.int64, device=self.dev)]
        col_parts, type_parts = [], []
        for q, r in enumerate(batch):
            row_parts.append(r.device["row_ptr"][1:] + int(nnz_off[q]))
            col_parts.append(r.device["col"] + int(node_off[q]))
            type_parts.append(r.device["types"])
        row_ptr = torch.cat(row_parts)
        col = torch.cat(col_parts) if col_parts else torch.zeros(0, dtype=torch.int32,
                                                                 device=self.dev)
        types = torch.cat(type_parts)
        gl = np.array([r.L for r in batch], dtype=np.int32)
        plan = BatchPlan(row_ptr, col.to(torch.int32), types, node_off, gl)
        glob, _ = count_batch(plan, workspace=ws, stream=stream)
        host = glob.cpu().numpy().view(np.uint64)
        return [host[plan.goff_host[q]:plan.goff_host[q + 1]].copy() for q in range(len(batch))]


def replay(server: Server, requests: list[Request], speed: float = 1.0) -> None:
    """Submit requests at their arrival times (seconds from now)."""
    start = server.now()
    for r in sorted(requests, key=lambda x: x.arrival):
        delay = start + r.arrival / speed - server.now()
        if delay > 0:
            time.sleep(delay)
        r.arrival = server.now()
        server.submit(r)
