"""Scheduling logic of the serving layer on the CPU, with a stand-in
backend (no GPU, no oracle).  Its 'device' runs each stream's steps one
after another on a fake clock that advances only when the server sleeps,
so arrival times, admission, overlap and latencies are all deterministic."""
import math

import numpy as np
import pytest

from paper_2604_09884_amd import configs
from paper_2604_09884_amd.serve import (ACTIVE, CANCELLED, DONE, FAILED, QUEUED, REFUSED,
                                        Request, Server, nearest_rank, poisson_arrivals)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """Request state lives in host arrays; a step moves theta towards the
    mean of y and reports a loss (non-finite if y holds a NaN).  A step of
    a request costs `cost` seconds of simulated device time (the problem's
    lr field is reused for nothing else); steps on one stream run in order,
    streams run concurrently.  Records creation order and live handles."""

    def __init__(self, clock, size=1000):
        self.clock, self.size = clock, size
        self.created, self.live = [], set()
        self.free_at = {}

    def reservation(self, req):
        return int(req.problem.N) * self.size

    def streams(self, n):
        return list(range(n))

    def create(self, req, stream):
        h = {"theta": np.asarray(req.theta0, dtype=np.float64).copy(),
             "y": np.asarray(req.y, dtype=np.float64), "lr": req.problem.lr,
             "cost": req.B if req.B is not None else 1.0}
        self.created.append(id(req))
        self.live.add(id(h))
        return h

    def launch(self, h, t, stream):
        g = h["theta"] - h["y"].mean() + 0.01 * (t + 1)
        h["theta"] -= h["lr"] * g
        start = max(self.clock(), self.free_at.get(stream, 0.0))
        self.free_at[stream] = start + h["cost"]
        return (self.free_at[stream], float(0.5 * (g * g).sum()))

    def ready(self, tok):
        return self.clock() >= tok[0]

    def read(self, tok):
        return tok[1], tok[1]

    def theta(self, h, stream):
        return h["theta"].copy()

    def release(self, h, stream):
        self.live.discard(id(h))


def _req(N, seed, steps=5, bad=False, cost=1.0):
    p = configs.C1.with_(N=N, lr=0.1)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(16)
    if bad:
        y[3] = np.nan
    return Request(problem=p, y=y, steps=steps, theta0=rng.standard_normal(8), B=cost)


def _server(budget=10 ** 9, **kw):
    clk = FakeClock()
    be = FakeBackend(clk)
    srv = Server(be, budget_bytes=budget, clock=clk, **kw)
    return srv, be, clk


def _run(srv, clk, limit=100000):
    n = 0
    while not srv.idle():
        if not srv.tick():
            clk.sleep(0.25)
        n += 1
        assert n < limit


def test_results_do_not_depend_on_the_mix():
    alone, _, ca = _server()
    ra = alone.submit(_req(16, 1, steps=4))
    _run(alone, ca)
    mixed, _, cm = _server(n_slots=2)
    ids = [mixed.submit(_req(16, s, steps=3 + s, cost=0.5 + s)) for s in (2, 1, 3)]
    _run(mixed, cm)
    assert alone.status(ra).state == DONE
    assert all(mixed.status(i).state == DONE for i in ids)
    assert np.array_equal(alone.status(ra).theta, mixed.status(ids[1]).theta)


def test_admission_by_budget_in_arrival_order():
    srv, be, clk = _server(budget=2 * 16 * 1000)   # two N=16 requests fit
    ids = [srv.submit(_req(16, s, steps=2 + s)) for s in range(4)]
    srv.tick()
    assert [srv.status(i).state for i in ids] == [ACTIVE, ACTIVE, QUEUED, QUEUED]
    peak = 0
    while not srv.idle():
        if not srv.tick():
            clk.sleep(0.25)
        peak = max(peak, len(srv.active()))
        assert srv.reserved <= srv.budget
    assert peak <= 2
    assert all(srv.status(i).state == DONE for i in ids)
    # creation followed arrival order
    assert be.created == [id(srv.status(i).req) for i in ids]
    assert srv.reserved == 0 and not be.live


def test_slots_bound_concurrency():
    srv, be, clk = _server(n_slots=3)
    ids = [srv.submit(_req(16, s, steps=3)) for s in range(7)]
    peak = 0
    while not srv.idle():
        if not srv.tick():
            clk.sleep(0.25)
        peak = max(peak, len(srv.active()))
    assert peak == 3 and all(srv.status(i).state == DONE for i in ids)


def test_requests_wait_for_their_arrival_time():
    srv, be, clk = _server()
    early = srv.submit(_req(16, 1, steps=2), arrival=0.0)
    late = srv.submit(_req(16, 2, steps=2), arrival=10.0)
    srv.tick()
    assert srv.status(early).state == ACTIVE and srv.status(late).state == QUEUED
    _run(srv, clk)
    s = srv.status(late)
    assert s.state == DONE and s.t_admit >= 10.0
    # latency is completion minus arrival: two 1-second steps, no queueing
    assert s.latency == pytest.approx(2.0, abs=0.3)
    assert srv.status(early).latency == pytest.approx(2.0, abs=0.3)


def test_short_requests_are_not_held_to_the_pace_of_long_ones():
    # one request with 10-second steps beside three with 1-second steps: the
    # short ones advance at their own rate and finish long before the long one
    srv, be, clk = _server(n_slots=4, depth=2)
    slow = srv.submit(_req(16, 0, steps=5, cost=10.0))
    fast = [srv.submit(_req(16, s, steps=5, cost=1.0)) for s in (1, 2, 3)]
    _run(srv, clk)
    for f in fast:
        assert srv.status(f).state == DONE and srv.status(f).latency < 6.0
    assert srv.status(slow).latency >= 50.0


def test_steps_stay_in_flight_per_request():
    # with depth 3, a request has three steps enqueued before any finishes
    srv, be, clk = _server(depth=3)
    r = srv.submit(_req(16, 1, steps=5, cost=1.0))
    srv.tick()
    s = srv.status(r)
    assert s.launched == 3 and s.step == 0 and len(s.inflight) == 3
    _run(srv, clk)
    assert s.state == DONE and s.step == 5 and s.launched == 5


def test_oversized_request_is_refused():
    srv, be, clk = _server(budget=16 * 1000)
    big = srv.submit(_req(64, 0))
    ok = srv.submit(_req(16, 1, steps=2))
    _run(srv, clk)
    assert srv.status(big).state == REFUSED and "exceeds" in srv.status(big).error
    assert srv.status(ok).state == DONE


def test_failure_is_isolated_and_memory_released():
    srv, be, clk = _server()
    good = srv.submit(_req(16, 1, steps=4))
    bad = srv.submit(_req(16, 2, steps=4, bad=True))
    _run(srv, clk)
    assert srv.status(bad).state == FAILED and "non-finite" in srv.status(bad).error
    assert srv.status(bad).step == 1
    assert srv.status(good).state == DONE
    ref, _, cr = _server()
    r = ref.submit(_req(16, 1, steps=4))
    _run(ref, cr)
    assert np.array_equal(srv.status(good).theta, ref.status(r).theta)
    assert srv.reserved == 0 and not be.live


def test_cancel_active_and_queued():
    srv, be, clk = _server(budget=16 * 1000)
    a = srv.submit(_req(16, 1, steps=10))
    b = srv.submit(_req(16, 2, steps=3))
    srv.tick()
    srv.cancel(b)          # still queued behind a
    srv.tick()
    srv.cancel(a)          # active
    assert srv.status(a).state == CANCELLED and srv.status(b).state == CANCELLED
    assert srv.idle() and srv.reserved == 0 and not be.live


def test_nearest_rank_percentiles():
    v = list(range(1, 65))          # 64 values
    assert nearest_rank(v, 50) == 32
    assert nearest_rank(v, 95) == 61
    assert nearest_rank(v, 99) == 64  # ceil(0.99 * 64) = 64: the maximum
    assert nearest_rank([3.0], 99) == 3.0
    assert math.isnan(nearest_rank([], 50))


def test_poisson_arrivals_are_seeded_and_have_the_rate():
    a = poisson_arrivals(64, 2.0, 5005)
    assert np.array_equal(a, poisson_arrivals(64, 2.0, 5005))
    assert np.all(np.diff(a) > 0) and a[0] > 0
    b = poisson_arrivals(20000, 2.0, 1)
    assert abs(np.mean(np.diff(b)) - 0.5) < 0.02


def test_metrics():
    srv, be, clk = _server()
    for s in range(3):
        srv.submit(_req(16, s, steps=2 + s), arrival=float(s))
    _run(srv, clk)
    m = srv.metrics()
    assert m["done"] == 3 and m["steps"] == 2 + 3 + 4
    assert m["latency_s_p99"] >= m["latency_s_p50"] > 0.0
    lat = sorted(srv.status(i).latency for i in range(3))
    assert m["latency_s_p50"] == lat[1] and m["latency_s_p99"] == lat[2]
    assert m["makespan_s"] > 0 and m["steps_per_s"] == pytest.approx(9 / m["makespan_s"])
