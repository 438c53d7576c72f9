"""Scheduler of the request loop on a CPU stand-in backend (no GPU)."""
import numpy as np
import pytest

from paper_1912_04064_amd import serving as S
from paper_1912_04064_amd import workloads as WL


class Req:
    def __init__(self, rid, arrival, n, steps):
        self.rid, self.arrival, self.n, self.steps = rid, arrival, n, steps


class FakeWl:
    def __init__(self, n):
        self.n_particles = n


def make(req):
    return FakeWl(req.n)


def mem(wl):
    return 1000 + wl.n_particles


def test_all_requests_complete_and_latency_covers_compute():
    reqs = [Req(i, 0.1 * i, 1000 * (1 + i % 3), 50 + 10 * (i % 4)) for i in range(20)]
    be = S.FakeBackend(rate=1e6, mem_fn=mem, max_runs=4)
    srv = S.Server(be, hbm_budget=10 ** 9, max_runs=4, steps_per_call=5)
    recs = srv.serve(reqs, make)
    assert len(recs) == 20 and all(np.isfinite(r.finished) for r in recs)
    for r, q in zip(recs, reqs):
        # a run alone would need steps * n / rate seconds
        assert r.latency >= q.steps * q.n / 1e6 - 1e-12
        assert r.admitted >= r.arrival and r.finished > r.admitted
        assert r.result["step"] == q.steps
    assert srv.max_active <= 4


def test_admission_respects_budget_and_slots():
    reqs = [Req(i, 0.0, 5000, 20) for i in range(10)]
    be = S.FakeBackend(rate=1e6, mem_fn=mem, max_runs=8)
    budget = 3 * mem(FakeWl(5000))            # room for three at a time
    srv = S.Server(be, hbm_budget=budget, max_runs=8, steps_per_call=4)
    live, peak = 0, 0
    recs = srv.serve(reqs, make)
    for t, ev, rid in sorted(srv.trace, key=lambda x: (x[0], x[1] == "admit")):
        live += 1 if ev == "admit" else -1
        peak = max(peak, live)
    assert peak <= 3 and srv.max_active <= 3
    assert len(recs) == 10


def test_continuous_batching_admits_while_others_run():
    """A short request arriving while a long one runs is admitted at once and
    finishes first: no waiting for the batch to drain."""
    reqs = [Req(0, 0.0, 10000, 1000), Req(1, 0.05, 1000, 10)]
    be = S.FakeBackend(rate=1e6, mem_fn=mem, max_runs=4)
    srv = S.Server(be, hbm_budget=10 ** 9, max_runs=4, steps_per_call=5)
    recs = srv.serve(reqs, make)
    long_run, short = recs
    assert short.admitted < long_run.finished
    assert short.finished < long_run.finished


def test_fifo_blocking_and_oversized_request():
    reqs = [Req(0, 0.0, 10 ** 6, 5)]
    be = S.FakeBackend(rate=1e6, mem_fn=mem, max_runs=4)
    srv = S.Server(be, hbm_budget=10 ** 5, max_runs=4)
    with pytest.raises(ValueError):
        srv.serve(reqs, make)


def test_request_stream_statistics():
    reqs = WL.request_stream(20.0, window_s=5.0, seed=5)
    lam = len(reqs) / 5.0
    assert 10 < lam < 30
    assert all(64 <= r.n[0] <= 1024 and 64 <= r.n[1] <= 256 for r in reqs)
    assert all(200 <= r.steps <= 2000 for r in reqs)
    gaps = np.diff([r.arrival for r in reqs])
    assert np.all(gaps > 0)


def test_summary_percentiles():
    recs = [S.RunRecord(i, 0.0, 0.0, float(i + 1), 10, 100, 1) for i in range(100)]
    s = S.summarize(recs)
    assert s["p50_latency_s"] == pytest.approx(50.5)
    assert s["p99_latency_s"] == pytest.approx(99.01)
    assert s["runs"] == 100
