"""The autotuner's search and its count checks, with a modelled clock and a
stand-in counting call (no GPU): coordinate descent must reach the modelled
optimum, keep the starting value on ties, and stop on differing counts."""

import pytest

from paper_2010_14058_amd import _lib
from paper_2010_14058_amd import autotune as AT


class Model:
    """A counting call whose duration is a function of the knobs in effect
    (read back from the library) and whose digest is fixed unless poisoned."""

    def __init__(self, cost, poison=None):
        self.cost = cost
        self.poison = poison
        self.now = 0.0
        self.calls = 0

    def clock(self):
        return self.now

    def run(self):
        knobs = _lib.get_tuning()
        self.calls += 1
        self.now += self.cost(knobs) / 1e3
        if self.poison and self.poison(knobs):
            return ("other",)
        return ("counts",)


@pytest.fixture
def restore_knobs():
    _lib.load()
    base = _lib.get_tuning()
    yield
    _lib.set_tuning(**base)


def test_descent_finds_separable_optimum(restore_knobs):
    def cost(k):
        return 100 + abs(k["light_wedges"] - 128) / 8 + abs(k["edge_deg"] - 64) / 4

    m = Model(cost)
    space = {"light_wedges": [64, 128, 256, 512], "edge_deg": [32, 64, 128, 1024]}
    res = AT.tune(m.run, space, repeats=2, clock=m.clock, log=None)
    assert res.best == {"light_wedges": 128, "edge_deg": 64}
    assert res.best_ms == pytest.approx(100.0)
    assert res.start_ms > res.best_ms
    # the thread's knobs are left at the best setting
    now = _lib.get_tuning()
    assert now["light_wedges"] == 128 and now["edge_deg"] == 64
    # each setting is timed once: the start and 3 + 3 trials in the first
    # round; the second retries light_wedges under the new edge_deg (3 new
    # settings), finds nothing better and stops
    assert len(res.trials) == 10


def test_small_gains_do_not_move(restore_knobs):
    _lib.set_tuning(light_wedges=512)

    def cost(k):
        return 100.0 - (0.5 if k["light_wedges"] == 256 else 0.0)

    m = Model(cost)
    res = AT.tune(m.run, {"light_wedges": [128, 256, 512]}, repeats=1, clock=m.clock, log=None,
                  min_gain=0.02)
    assert res.best == {"light_wedges": 512}


def test_mismatching_counts_raise(restore_knobs):
    m = Model(lambda k: 10.0, poison=lambda k: k["edge_deg"] == 128)
    with pytest.raises(AT.MismatchError):
        AT.tune(m.run, {"edge_deg": [1024, 256, 128]}, repeats=1, clock=m.clock, log=None)


def test_profile_roundtrip(tmp_path, restore_knobs):
    res = AT.TuneResult(best={"light_wedges": 256, "edge_deg": 512}, best_ms=1.0, start_ms=2.0)
    path = str(tmp_path / "p.json")
    AT.save(res, path, "unit")
    prof = AT.load(path)
    assert prof["workload"] == "unit" and prof["knobs"] == res.best
    AT.apply(prof)
    now = _lib.get_tuning()
    assert now["light_wedges"] == 256 and now["edge_deg"] == 512
    with pytest.raises(ValueError):
        AT.tune(lambda: 0, {"no_such_knob": [1]}, log=None)


def test_shipped_profiles_apply(restore_knobs):
    """Every profile under paper_2010_14058_amd/tuned/ names its workload,
    holds only known knobs, and is accepted by the library as it stands."""
    import glob
    import os

    d = os.path.join(os.path.dirname(AT.__file__), "tuned")
    paths = sorted(glob.glob(os.path.join(d, "*.json")))
    assert paths
    for p in paths:
        prof = AT.load(p)
        assert prof["workload"] == os.path.basename(p)[:-5]
        AT.apply(prof)
        now = _lib.get_tuning()
        for k, v in prof["knobs"].items():
            assert now[k] == v, (p, k)
        assert prof["best_ms"] <= prof["start_ms"]
