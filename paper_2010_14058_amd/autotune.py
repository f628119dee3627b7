"""Autotuner for the library's scheduling knobs on one workload.

The knobs of ``tg_set_tuning`` decide how work is cut and scheduled (task
sizes, workgroup counts, the degree buckets that send 4-cycle groups and
edges to the one-wave or the workgroup kernels); they never change a count.
The tuner searches them by coordinate descent: each knob in turn takes every
candidate value while the others stay fixed, a value replaces the current one
only when its time is lower by more than ``min_gain``, and rounds repeat until
a round changes nothing (or ``rounds`` is reached).  A setting is timed as the
median of ``repeats`` calls after one untimed call.

Because the counts are exact integers, every call of every setting must give
the same result: ``run`` returns a digest of its output and the tuner raises
``MismatchError`` as soon as a digest differs from the first one.

Profiles are JSON files (``save`` / ``load``) holding the knob values and
the workload they were tuned on; ``apply`` sets them for the calling thread.
"""

from __future__ import annotations

import json
import statistics
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Sequence

from . import _lib

# Candidate values.  Single graphs: the heavy 4-cycle task size and clear
# threshold, the heavy workgroup counts, the light-kernel derivation batch
# and both degree buckets.  Batches of small graphs: the degree buckets and
# the heavy workgroup counts (a batch derives edge by edge).
SINGLE_SPACE: Dict[str, List[int]] = {
    "task_wedges": [1 << 16, 1 << 17, 1 << 18, 1 << 19],
    "clear_bytes": [0, 16, 64, 256],
    "cycle_slots": [512, 1024, 1536, 2048],
    "edge_slots": [512, 1024, 1280, 1536, 2048],
    "derive_edges": [0, 1, 2, 3],
    "light_wedges": [128, 256, 512],
    "edge_deg": [512, 640, 768, 832, 896, 1024],
}
BATCH_SPACE: Dict[str, List[int]] = {
    "light_wedges": [64, 128, 256, 512],
    "edge_deg": [32, 64, 128, 256, 1024],
    "cycle_slots": [256, 512, 1024],
    "task_wedges": [1 << 16, 1 << 18, 1 << 20],
}


class MismatchError(RuntimeError):
    """Two settings of the scheduling knobs gave different counts."""


@dataclass
class TuneResult:
    best: Dict[str, int]
    best_ms: float
    start_ms: float
    trials: List[dict] = field(default_factory=list)

    def to_json(self, workload: str) -> dict:
        return {"workload": workload, "knobs": dict(self.best), "best_ms": round(self.best_ms, 3),
                "start_ms": round(self.start_ms, 3), "trials": self.trials}


def _time_setting(run: Callable[[], object], knobs: Dict[str, int], repeats: int,
                  clock: Callable[[], float], expect, log) -> tuple:
    _lib.set_tuning(**knobs)
    digest = run()  # untimed: workspace growth, caches
    if expect is not None and digest != expect:
        raise MismatchError(f"counts differ under {knobs}")
    times = []
    for _ in range(repeats):
        t0 = clock()
        d = run()
        times.append((clock() - t0) * 1e3)
        if d != digest:
            raise MismatchError(f"counts differ between calls under {knobs}")
    ms = statistics.median(times)
    if log:
        log(f"  {knobs} -> {ms:.2f} ms")
    return ms, digest


def tune(run: Callable[[], object], space: Dict[str, Sequence[int]], *, repeats: int = 3,
         rounds: int = 2, min_gain: float = 0.02, clock: Callable[[], float] = time.perf_counter,
         log: Callable[[str], None] | None = print) -> TuneResult:
    """Coordinate descent over ``space`` (knob -> candidate values).

    ``run`` performs one complete counting call (returning when the counts
    are done) and returns a digest of its output.  The knobs in effect when
    ``tune`` is called are the starting point; the thread's knobs are left
    at the best setting found.
    """
    for name in space:
        if name not in _lib.TUNE_KNOBS:
            raise ValueError(f"unknown knob {name}")
    current = {k: v for k, v in _lib.get_tuning().items() if k in space}
    cache: Dict[tuple, float] = {}
    trials: List[dict] = []
    expect = None

    def timed(knobs):
        nonlocal expect
        key = tuple(sorted(knobs.items()))
        if key not in cache:
            ms, digest = _time_setting(run, knobs, repeats, clock, expect, log)
            if expect is None:
                expect = digest
            cache[key] = ms
            trials.append({"knobs": dict(knobs), "ms": round(ms, 3)})
        return cache[key]

    start_ms = best_ms = timed(current)
    for _ in range(rounds):
        changed = False
        for name, values in space.items():
            for v in values:
                if v == current[name]:
                    continue
                trial = dict(current, **{name: v})
                ms = timed(trial)
                if ms < best_ms * (1.0 - min_gain):
                    current, best_ms, changed = trial, ms, True
        if not changed:
            break
    _lib.set_tuning(**current)
    return TuneResult(best=current, best_ms=best_ms, start_ms=start_ms, trials=trials)


def save(result: TuneResult, path: str, workload: str) -> None:
    with open(path, "w") as f:
        json.dump(result.to_json(workload), f, indent=1)
        f.write("\n")


def load(path: str) -> dict:
    with open(path) as f:
        prof = json.load(f)
    for name in prof["knobs"]:
        if name not in _lib.TUNE_KNOBS:
            raise ValueError(f"unknown knob {name} in {path}")
    return prof


def apply(profile: dict) -> dict:
    """Set a profile's knobs for this thread; returns the previous values."""
    return _lib.set_tuning(**profile["knobs"])


def digest_of(glob, rows=None) -> tuple:
    """Exact digest of one call's results, computed on the device: for the
    global vector (or a batch's concatenated vectors) its length, its sum and
    its index-weighted sum (wrapping int64); for a per-edge table its column
    sums."""
    import torch

    g = None
    if glob is not None:
        flat = glob.reshape(-1)
        idx = torch.arange(1, flat.numel() + 1, dtype=torch.int64, device=flat.device)
        g = (flat.numel(), int(flat.sum().item()), int((flat * idx).sum().item()))
    r = tuple(rows.sum(dim=0).tolist()) if rows is not None else None
    return g, r
