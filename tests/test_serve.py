"""Scheduling logic of the serving layer on the CPU, with a stand-in
backend whose 'step' is a deterministic update (no GPU, no oracle)."""
import math

import numpy as np
import pytest

from paper_2604_09884_amd import configs
from paper_2604_09884_amd.serve import (CANCELLED, DONE, FAILED, REFUSED, Request, Server)


class FakeBackend:
    """Request state lives in host arrays; a step moves theta towards the
    mean of y and reports a loss.  A request whose y holds a NaN produces a
    non-finite loss.  Records creation order and live handles."""

    def __init__(self, size=1000):
        self.size = size
        self.created, self.live = [], set()

    def reservation(self, req):
        return int(req.problem.N) * self.size

    def create(self, req):
        h = {"theta": np.asarray(req.theta0, dtype=np.float64).copy(),
             "y": np.asarray(req.y, dtype=np.float64), "lr": req.problem.lr, "id": id(req)}
        self.created.append(id(req))
        self.live.add(id(h))
        return h

    def step(self, h, t, stream):
        g = h["theta"] - h["y"].mean() + 0.01 * (t + 1)
        h["theta"] -= h["lr"] * g
        h["loss"] = float(0.5 * (g * g).sum())

    def streams(self, n):
        return list(range(n))

    def sync(self, streams):
        pass

    def read(self, h):
        return h["loss"], h["loss"]

    def theta(self, h):
        return h["theta"].copy()

    def release(self, h):
        self.live.discard(id(h))


def _req(N, seed, steps=5, bad=False):
    p = configs.C1.with_(N=N, lr=0.1)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(16)
    if bad:
        y[3] = np.nan
    return Request(problem=p, y=y, steps=steps, theta0=rng.standard_normal(8))


def test_results_do_not_depend_on_the_mix():
    alone = Server(FakeBackend(), budget_bytes=10 ** 9)
    ra = alone.submit(_req(16, 1, steps=4))
    alone.run()
    mixed = Server(FakeBackend(), budget_bytes=10 ** 9, n_streams=2)
    ids = [mixed.submit(_req(16, s, steps=3 + s)) for s in (2, 1, 3)]
    mixed.run()
    assert alone.status(ra).state == DONE
    assert all(mixed.status(i).state == DONE for i in ids)
    assert np.array_equal(alone.status(ra).theta, mixed.status(ids[1]).theta)


def test_admission_by_budget_in_arrival_order():
    be = FakeBackend()
    srv = Server(be, budget_bytes=2 * 16 * be.size)   # two N=16 requests fit
    ids = [srv.submit(_req(16, s, steps=2 + s)) for s in range(4)]
    srv.tick()
    assert [srv.status(i).state for i in ids] == ["active", "active", "queued", "queued"]
    peak = 0
    while not srv.idle():
        srv.tick()
        peak = max(peak, len(srv.active()))
        assert srv.reserved <= srv.budget
    assert peak <= 2
    assert all(srv.status(i).state == DONE for i in ids)
    # creation followed arrival order
    assert be.created == [id(srv.status(i).req) for i in ids]
    assert srv.reserved == 0 and not be.live


def test_oversized_request_is_refused():
    be = FakeBackend()
    srv = Server(be, budget_bytes=16 * be.size)
    big = srv.submit(_req(64, 0))
    ok = srv.submit(_req(16, 1, steps=2))
    srv.run()
    assert srv.status(big).state == REFUSED and "exceeds" in srv.status(big).error
    assert srv.status(ok).state == DONE


def test_failure_is_isolated_and_memory_released():
    be = FakeBackend()
    srv = Server(be, budget_bytes=10 ** 9)
    good = srv.submit(_req(16, 1, steps=4))
    bad = srv.submit(_req(16, 2, steps=4, bad=True))
    srv.run()
    assert srv.status(bad).state == FAILED and "non-finite" in srv.status(bad).error
    assert srv.status(bad).step == 1
    assert srv.status(good).state == DONE
    ref = Server(FakeBackend(), budget_bytes=10 ** 9)
    r = ref.submit(_req(16, 1, steps=4))
    ref.run()
    assert np.array_equal(srv.status(good).theta, ref.status(r).theta)
    assert srv.reserved == 0 and not be.live


def test_cancel_active_and_queued():
    be = FakeBackend()
    srv = Server(be, budget_bytes=16 * be.size)
    a = srv.submit(_req(16, 1, steps=10))
    b = srv.submit(_req(16, 2, steps=3))
    srv.tick()
    srv.cancel(b)          # still queued behind a
    srv.tick()
    srv.cancel(a)          # active
    assert srv.status(a).state == CANCELLED and srv.status(b).state == CANCELLED
    assert srv.idle() and srv.reserved == 0 and not be.live


def test_metrics():
    srv = Server(FakeBackend(), budget_bytes=10 ** 9)
    for s in range(3):
        srv.submit(_req(16, s, steps=2 + s))
    srv.run()
    m = srv.metrics()
    assert m["done"] == 3 and m["steps"] == 2 + 3 + 4
    assert m["tick_ms_p99"] >= m["tick_ms_p50"] >= 0.0
    assert math.isfinite(m["tick_ms_p99"])
