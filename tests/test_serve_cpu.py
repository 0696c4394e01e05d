"""Scheduler of the serving loop on a simulated device (CPU only):
admission by footprint, back-pressure, FIFO order, completion and latency
accounting."""
import numpy as np
import pytest

from paper_2106_03872_amd import serve, synth


def _trace(n=40, seed=5, rate=200.0):
    reqs = []
    for i, (t, spec) in enumerate(synth.serving_trace(n, rate, seed)):
        reqs.append(serve.Request(rid=i, arrival=t, spec=spec, nsteps=5))
    return reqs


def test_all_requests_complete_within_budget():
    reqs = _trace()
    be = serve.FakeBackend(lanes=4)
    budget = 3 * max(be.footprint(r) for r in reqs)
    srv = serve.Server(be, budget)
    done = srv.run(reqs)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert srv.max_used <= budget
    assert all(len(r.step_times) == 5 for r in done)
    assert all(np.all(np.diff([r.t_admit] + r.step_times) > 0) for r in done)
    # admission is first-come first-served
    assert be.admitted == sorted(be.admitted, key=lambda i: (reqs[i].arrival, i))
    rep = serve.Server.report(done, srv.elapsed, serve.hpsi_per_step)
    assert rep["requests"] == len(reqs) and rep["steps"] == 5 * len(reqs)
    assert rep["step_latency_ms_p99"] >= rep["step_latency_ms_p50"] > 0
    assert rep["orbital_hpsi_per_s"] > 0


def test_backpressure_limits_concurrency():
    reqs = _trace(20)
    be = serve.FakeBackend(lanes=2, footprint_fn=lambda r: 100)
    srv = serve.Server(be, hbm_budget=250)         # at most two resident requests
    done = srv.run(reqs)
    assert srv.max_used <= 250 and len(done) == 20
    # intervals [admission start, done] never overlap more than twice
    ev = sorted([(r.t_submit, 1) for r in done] + [(r.t_done, -1) for r in done], key=lambda x: (x[0], x[1]))
    level = 0
    for _, d in ev:
        level += d
        assert level <= 2


def test_request_larger_than_budget_is_rejected():
    reqs = _trace(3)
    be = serve.FakeBackend(footprint_fn=lambda r: 10 ** 12)
    with pytest.raises(ValueError):
        serve.Server(be, hbm_budget=10 ** 9).run(reqs)


def test_more_lanes_finish_sooner():
    t1 = serve.Server(serve.FakeBackend(lanes=1), 10 ** 13)
    t1.run(_trace(30))
    t4 = serve.Server(serve.FakeBackend(lanes=4), 10 ** 13)
    t4.run(_trace(30))
    assert t4.elapsed < t1.elapsed


def test_failing_requests_fail_alone():
    reqs = _trace(24)
    be = serve.FakeBackend(lanes=3, fail_admit={3, 11}, fail_step={7}, fail_retire={15})
    budget = 4 * max(be.footprint(r) for r in reqs)
    srv = serve.Server(be, budget)
    done = srv.run(reqs)
    failed = {r.rid for r in srv.failed}
    assert failed == {3, 7, 11, 15}
    assert sorted(r.rid for r in done) == sorted(set(range(24)) - failed)
    assert all(len(r.step_times) == 5 and not r.error for r in done)
    assert all(r.error for r in srv.failed)
    assert 7 in be.discarded                       # the failed step's request was freed
    assert srv.used_at_end == 0                    # every reservation was released


def test_memory_short_admission_is_retried():
    reqs = _trace(20)
    be = serve.FakeBackend(lanes=3, short_once={2, 9})
    srv = serve.Server(be, 6 * max(be.footprint(r) for r in reqs))
    done = srv.run(reqs)
    assert not srv.failed and sorted(r.rid for r in done) == list(range(20))
    assert srv.requeued == 2
    assert be.admitted.count(2) == 2 and be.admitted.count(9) == 2
    assert srv.used_at_end == 0
