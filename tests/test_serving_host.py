"""Host logic of the request server, without a GPU: admission by slots and
HBM budget in arrival order, a request larger than the budget still served
alone, per-request errors, and the latency summary.  The problem solve is
replaced by a timed stand-in that records what ran concurrently."""
import threading
import time
from dataclasses import dataclass

import numpy as np
import pytest

from paper_2008_02205_amd import mlpg
from paper_2008_02205_amd.serving import Result, Server, hbm_estimate, latency_summary


@dataclass
class Spec:
    rid: int
    arrival: float
    side: int
    n_ord: int
    secs: float = 0.05
    fail: bool = False


class _Recorder(Server):
    """Server whose solve sleeps and records the requests running at once."""

    def __init__(self, slots, budget):
        self.slots, self.budget, self.precision, self.opts = slots, budget, mlpg.MLPG_MIXED, None
        self.lock = threading.Lock()
        self.running = {}
        self.snapshots = []
        self.starts = []

    def _stream(self):
        return None

    def _solve(self, build, spec, stream, true_up=None):
        need = hbm_estimate(spec.side * spec.side, spec.n_ord, self.precision)
        with self.lock:
            self.running[spec.rid] = need
            self.snapshots.append(dict(self.running))
            self.starts.append(spec.rid)
        try:
            time.sleep(spec.secs)
            if spec.fail:
                raise RuntimeError("stand-in failure")
            return np.full(3, spec.rid, float), np.zeros(3), {"converged": 1}
        finally:
            with self.lock:
                del self.running[spec.rid]


def _need(side, n_ord):
    return hbm_estimate(side * side, n_ord, mlpg.MLPG_MIXED)


def test_slots_and_budget_bound_what_runs_together():
    specs = [Spec(i, 0.0, side, n_ord) for i, (side, n_ord) in
             enumerate([(64, 32), (96, 64), (32, 16), (128, 64), (48, 32), (80, 16), (64, 64), (40, 32)])]
    budget = _need(96, 64) + _need(64, 32)   # about two mid-size problems at a time
    srv = _Recorder(slots=3, budget=budget)
    res = srv.run(specs, build=None, realtime=False)
    assert [r.rid for r in res] == list(range(len(specs)))
    assert all(r.error is None and r.info["converged"] == 1 for r in res)
    for snap in srv.snapshots:
        assert len(snap) <= 3
        if len(snap) > 1:
            assert sum(snap.values()) <= budget
    assert max(len(s) for s in srv.snapshots) >= 2   # the budget does allow overlap


def test_first_fit_in_arrival_order_and_an_oversize_request_runs_alone():
    big = Spec(0, 0.0, 256, 128, secs=0.05)
    small = [Spec(i, 0.0, 32, 16, secs=0.05) for i in range(1, 4)]
    budget = _need(32, 16) * 2 + 1          # the big request alone exceeds it
    assert _need(256, 128) > budget
    srv = _Recorder(slots=4, budget=budget)
    res = srv.run([big] + small, build=None, realtime=False)
    assert all(r.error is None for r in res)
    assert srv.starts[0] == 0                          # first in arrival order, admitted alone
    first = srv.snapshots[0]
    assert list(first) == [0]
    for snap in srv.snapshots:
        if 0 in snap:
            assert len(snap) == 1                      # nothing joins the oversize request
    assert srv.starts[1:] == [1, 2, 3]                 # the rest in arrival order


def test_arrivals_in_real_time_and_errors_per_request():
    specs = [Spec(0, 0.00, 32, 16, secs=0.02), Spec(1, 0.05, 32, 16, secs=0.02, fail=True),
             Spec(2, 0.10, 32, 16, secs=0.02)]
    srv = _Recorder(slots=2, budget=_need(32, 16) * 4)
    res = srv.run(specs, build=None, realtime=True)
    assert res[1].error is not None and "stand-in failure" in res[1].error
    assert res[0].error is None and res[2].error is None
    for r, s in zip(res, specs):
        assert r.admitted >= s.arrival - 1e-3          # nothing starts before it arrives
        assert r.done >= r.admitted
    summ = latency_summary(res)
    assert summ["requests"] == 3 and summ["failed"] == 1
    lat = sorted(r.latency for r in res if r.error is None)
    assert summ["p50_s"] == pytest.approx(float(np.percentile(lat, 50)))
    assert summ["p99_s"] == pytest.approx(float(np.percentile(lat, 99)))


def test_latency_summary_by_hand():
    rs = [Result(0, 0.0, 0.0, 1.0), Result(1, 0.5, 0.5, 2.5), Result(2, 1.0, 1.0, 4.0),
          Result(3, 1.0, 1.0, 9.0, error="x")]
    summ = latency_summary(rs)
    assert summ["failed"] == 1 and summ["requests"] == 4
    assert summ["p50_s"] == pytest.approx(2.0)          # latencies 1, 2, 3
    assert summ["mean_s"] == pytest.approx(2.0)
    assert summ["throughput_req_s"] == pytest.approx(4 / 9.0)


class _TrueUp(_Recorder):
    """Stand-in whose exact footprint (reported after 'assembly') is a quarter of the bound."""

    def _solve(self, build, spec, stream, true_up=None):
        if true_up is not None:
            true_up(hbm_estimate(spec.side * spec.side, spec.n_ord, self.precision) // 4)
        return super()._solve(build, spec, stream)


def test_exact_bytes_replace_the_reservation():
    """Once a running request reports its exact bytes, the freed part of its bound admits the
    next request while it still runs; the bytes return to zero at the end."""
    specs = [Spec(0, 0.0, 64, 64, secs=0.2), Spec(1, 0.0, 64, 64, secs=0.05)]
    budget = _need(64, 64) + _need(64, 64) // 2       # two bounds do not fit, bound + exact do
    srv = _TrueUp(slots=2, budget=budget)
    res = srv.run(specs, build=None, realtime=False)
    assert all(r.error is None for r in res)
    assert any(len(snap) == 2 for snap in srv.snapshots)   # they overlapped
    assert all(r.exact_bytes == _need(64, 64) // 4 for r in res)
    summ = latency_summary(res)
    assert summ["exact_over_reserved"] == pytest.approx(0.25, rel=1e-6)
