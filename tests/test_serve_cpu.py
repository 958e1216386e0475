"""Serving scheduler with the deterministic CPU executor: admission by
device footprint, eviction, continuous batching and latency bookkeeping."""
import numpy as np

from paper_2008_01539_amd.serve import FakeExecutor, Request, Server, SessionSpec


def _specs(k, fp=100):
    return [SessionSpec(name=f"s{i}", model=None, options=None,
                        schedule=np.array([1.0, 2.0, 4.0])) for i in range(k)]


def test_requests_join_while_others_run():
    ex = FakeExecutor(iter_cost=1.0, per_member=0.0,
                      iters_per_step=lambda s, k: 5 if s == "s0" else 2)
    srv = Server(_specs(3), ex, budget_bytes=10 ** 9, max_inflight=8, footprint=lambda s: 10)
    srv.submit(Request(0, 0, arrival=0.0))
    srv.tick()
    srv.tick()
    # a request for another session arrives while s0 is still iterating
    srv.submit(Request(1, 1, arrival=ex.now()))
    srv.tick()
    assert len(srv.inflight) == 2          # it joined at the next tick
    while srv.inflight:
        srv.tick()
    r0, r1 = sorted(srv.done, key=lambda r: r.rid)
    assert r1.finish < r0.finish           # the late, short request left first
    assert ex.ticks == [1, 1, 2, 2, 1]


def test_one_request_per_session_in_order():
    ex = FakeExecutor(iter_cost=1.0, per_member=0.0)
    srv = Server(_specs(1), ex, budget_bytes=10 ** 9, footprint=lambda s: 1)
    for k in range(3):
        srv.submit(Request(k, 0, arrival=0.0))
    while srv.queue or srv.inflight:
        srv.tick()
    assert [r.rid for r in srv.done] == [0, 1, 2]
    assert [r.step_index for r in srv.done] == [0, 1, 2]
    assert [r.dt for r in srv.done] == [1.0, 2.0, 4.0]
    assert all(r.arrival <= r.start <= r.finish for r in srv.done)


def test_admission_by_footprint_evicts_idle_sessions():
    ex = FakeExecutor(iter_cost=1.0, per_member=0.0, iters_per_step=lambda s, k: 2)
    srv = Server(_specs(4), ex, budget_bytes=250, max_inflight=8, footprint=lambda s: 100)
    for k in range(4):
        srv.submit(Request(k, k, arrival=0.0))
    srv.tick()
    assert len(srv.inflight) == 2 and srv.used == 200   # only two fit
    while srv.queue or srv.inflight:
        srv.tick()
        assert srv.used <= 250
    assert srv.stats.completed == 4
    assert srv.stats.evictions >= 2


def test_max_inflight_and_poisson_statistics():
    ex = FakeExecutor(iter_cost=0.01, per_member=0.001, iters_per_step=lambda s, k: 3)
    srv = Server(_specs(6), ex, budget_bytes=10 ** 9, max_inflight=4, footprint=lambda s: 1)
    summ = srv.run_poisson(rate=50.0, duration=5.0, mix=np.full(6, 1 / 6), seed=3)
    assert max(ex.ticks) <= 4
    assert summ["completed"] == len(srv.done)
    assert summ["completed"] > 150
    assert 0 < summ["p50_ms"] <= summ["p99_ms"]
    lat = np.array(srv.stats.latencies)
    assert np.all(lat > 0)
