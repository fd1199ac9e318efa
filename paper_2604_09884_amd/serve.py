"""Serving: many CT reconstructions stepped concurrently on one GPU.

Each request is one reconstruction problem: a geometry, its sinogram y, an
INR architecture and optimiser settings, and a number of gradient steps
(Algorithm 1 followed by Adam).  From admission to retirement its
parameters, Adam state, data and every scratch buffer stay resident on the
device.

Scheduling is continuous, not lock-step.  Requests arrive on a clock (each
has an arrival time; `submit` without one arrives at once).  An arrived
request is admitted, in arrival order, as soon as a slot is free and its
device bytes fit the budget.  Every active request owns one HIP stream of a
pool and keeps up to `depth` of its own steps in flight there; after each
step the loss and gradient norm are copied to pinned host memory behind an
event.  The scheduler polls those events: a request advances as fast as its
own steps finish, so short 2D requests are not held back by long 3D ones,
and the steps of different requests overlap on the device.  No step waits
for another request's step, and the host never synchronises the device
while requests run.

Per-request results do not depend on the mix: each request owns its
buffers, the step kernels use no atomics and reduce in a fixed order, and
requests share nothing but the device.

Admission is by device memory.  A request's bytes come from the library's
own sizing (`ops.request_device_bytes`, i.e. inrct_workspace_bytes for its
three handles plus the tensors the caller owns); a request that can never
fit is refused.  A request whose loss or gradient norm turns non-finite, or
whose launch raises, is retired as failed and its memory released; the
others keep running.  Requests can be cancelled at any time.

The scheduler is host logic over a backend object.  `HipBackend` drives
the C ABI through `ops` (there is no other product backend; tests supply
their own stand-in to exercise the scheduling logic on the CPU).
"""
from __future__ import annotations

import collections
import dataclasses
import itertools
import math
import time
from typing import Any, Deque, Dict, List, Optional

import numpy as np

from .configs import Problem


@dataclasses.dataclass
class Request:
    """One reconstruction.  `y` is the sinogram (host array or device
    tensor, view-major); `theta0` the initial parameters (None: seeded init
    from the problem)."""
    problem: Problem
    y: Any
    steps: int
    theta0: Any = None
    B: Any = None
    mlp_dtype: Optional[str] = None
    v_mode: str = "full"


QUEUED, ACTIVE, DONE, FAILED, CANCELLED, REFUSED = (
    "queued", "active", "done", "failed", "cancelled", "refused")


@dataclasses.dataclass
class Slot:
    rid: int
    req: Request
    state: str = QUEUED
    handle: Any = None
    stream: Any = None
    reserved: int = 0
    launched: int = 0      # steps enqueued
    step: int = 0          # steps finished and checked
    loss: float = math.nan
    gnorm2: float = math.nan
    error: str = ""
    t_arrive: float = 0.0  # seconds on the server clock
    t_admit: float = math.nan
    t_end: float = math.nan
    theta: Any = None      # final parameters (host copy) once done
    inflight: Deque[Any] = dataclasses.field(default_factory=collections.deque)

    @property
    def latency(self) -> float:
        """Completion minus arrival (seconds)."""
        return self.t_end - self.t_arrive


def nearest_rank(values, q: float) -> float:
    """The q-th percentile by the nearest-rank rule: the smallest value with
    at least q% of the values at or below it."""
    v = sorted(values)
    if not v:
        return math.nan
    return float(v[max(1, math.ceil(q / 100.0 * len(v))) - 1])


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process: cumulative sums of exponential
    gaps with mean 1/rate, from a seeded generator."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=n)
    return np.cumsum(gaps)


class HipBackend:
    """Creates a request's device state through `ops` on the request's own
    stream, enqueues its steps there, and reports each step's loss and
    gradient norm through pinned host memory behind an event."""

    RING = 8  # pinned result slots per request (more than any depth)

    def __init__(self, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)

    def reservation(self, req: Request) -> int:
        from . import lib as L
        from . import ops
        v_mode = L.INRCT_V_FULL if req.v_mode == "full" else L.INRCT_V_AT_I
        return ops.request_device_bytes(req.problem, req.mlp_dtype, v_mode)

    def streams(self, n: int):
        return [self.torch.cuda.Stream(device=self.device) for _ in range(n)]

    def create(self, req: Request, stream):
        from . import lib as L
        from . import ops, synth
        torch = self.torch
        p = req.problem
        dtype = req.mlp_dtype or p.mlp_dtype
        if req.theta0 is None:
            theta, B = synth.init_inr(p.arch, p.seed_init)
        else:
            theta, B = req.theta0, req.B
        with torch.cuda.stream(stream):
            th = torch.as_tensor(np.asarray(theta, dtype=np.float32) if not torch.is_tensor(theta)
                                 else theta, dtype=torch.float32, device=self.device).clone()
            Bv = (np.zeros(1, np.float32) if B is None or np.size(B) == 0
                  else np.asarray(B).ravel())
            Bd = torch.as_tensor(Bv, dtype=torch.float32, device=self.device)
            yd = torch.as_tensor(np.asarray(req.y, dtype=np.float32).ravel()
                                 if not torch.is_tensor(req.y) else req.y.reshape(-1),
                                 dtype=torch.float32, device=self.device)
            model = ops.Model(p.arch, p.dim, p.N, dtype, max_k=p.k())
            geom = ops.Geometry(p)
            k = p.k(model.n_fov)
            v_mode = L.INRCT_V_FULL if req.v_mode == "full" else L.INRCT_V_AT_I
            st = ops.GradStepper(model, geom, th, Bd, yd, k, p.lr, seed=p.seed_sampler,
                                 v_mode=v_mode)
            ring = torch.zeros((self.RING, 2), dtype=torch.float64, pin_memory=True)
        return {"stepper": st, "model": model, "geom": geom, "ring": ring, "next": 0}

    def launch(self, h, t: int, stream):
        """Enqueues step t; returns a token for `ready` / `read`."""
        torch = self.torch
        st = h["stepper"]
        slot = h["ring"][h["next"] % self.RING]
        h["next"] += 1
        with torch.cuda.stream(stream):
            st.step(t)
            slot.copy_(st.stats, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev, slot

    def ready(self, token) -> bool:
        return token[0].query()

    def read(self, token):
        return float(token[1][0]), float(token[1][1])

    def theta(self, h, stream):
        stream.synchronize()
        return h["stepper"].theta.detach().cpu().numpy()

    def release(self, h, stream):
        # the request's kernels must be done before its memory goes back
        stream.synchronize()
        h["stepper"].close()
        h["model"].close()
        h["geom"].close()
        h.clear()


class Server:
    """Continuous batching of gradient steps over resident requests."""

    def __init__(self, backend=None, budget_bytes: Optional[int] = None, n_slots: int = 8,
                 depth: int = 2, clock=time.perf_counter):
        self.backend = backend if backend is not None else HipBackend()
        if budget_bytes is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(free * 0.8)
        self.budget = int(budget_bytes)
        self.depth = max(1, int(depth))
        self.reserved = 0
        self.slots: Dict[int, Slot] = {}
        self.queue: List[int] = []          # arrival order (submitted, not admitted)
        self._ids = itertools.count()
        self._clock = clock
        self.t0 = clock()
        self.free_streams = self.backend.streams(max(1, n_slots))
        self.n_slots = len(self.free_streams)
        self.ticks = 0
        self.t_first_admit = math.nan
        self.t_last_end = math.nan

    def now(self) -> float:
        return self._clock() - self.t0

    # ---- requests
    def submit(self, req: Request, arrival: Optional[float] = None) -> int:
        """Adds a request that arrives at `arrival` seconds on the server
        clock (now if None)."""
        rid = next(self._ids)
        s = Slot(rid, req, t_arrive=self.now() if arrival is None else float(arrival))
        s.reserved = int(self.backend.reservation(req))
        self.slots[rid] = s
        if s.reserved > self.budget:
            s.state, s.error = REFUSED, "reservation %d B exceeds the budget %d B" % (
                s.reserved, self.budget)
            s.t_end = max(self.now(), s.t_arrive)
        else:
            self.queue.append(rid)
            self.queue.sort(key=lambda i: (self.slots[i].t_arrive, i))
        return rid

    def cancel(self, rid: int):
        s = self.slots[rid]
        if s.state == QUEUED:
            self.queue.remove(rid)
            s.state, s.t_end = CANCELLED, self.now()
        elif s.state == ACTIVE:
            self._retire(s, CANCELLED)

    def status(self, rid: int) -> Slot:
        return self.slots[rid]

    def active(self) -> List[Slot]:
        return [s for s in self.slots.values() if s.state == ACTIVE]

    def idle(self) -> bool:
        return not self.queue and not self.active()

    # ---- scheduling
    def _admit(self, now: float):
        while self.queue and self.free_streams:
            s = self.slots[self.queue[0]]
            if s.t_arrive > now or self.reserved + s.reserved > self.budget:
                break  # arrival order: later requests wait behind this one
            self.queue.pop(0)
            stream = self.free_streams.pop(0)
            try:
                s.handle = self.backend.create(s.req, stream)
            except Exception as e:  # creation failed: nothing stays reserved
                self.free_streams.append(stream)
                s.state, s.error, s.t_end = FAILED, "create: %s" % e, self.now()
                continue
            s.stream = stream
            self.reserved += s.reserved
            s.state, s.t_admit = ACTIVE, self.now()
            if math.isnan(self.t_first_admit):
                self.t_first_admit = s.t_admit

    def _retire(self, s: Slot, state: str, error: str = ""):
        try:
            if state == DONE:
                s.theta = self.backend.theta(s.handle, s.stream)
            self.backend.release(s.handle, s.stream)
        finally:
            s.handle = None
            s.inflight.clear()
            self.free_streams.append(s.stream)
            s.stream = None
            self.reserved -= s.reserved
            s.state, s.error, s.t_end = state, error, self.now()
            if state == DONE:
                self.t_last_end = s.t_end if math.isnan(self.t_last_end) else max(
                    self.t_last_end, s.t_end)

    def _launch(self, s: Slot):
        while len(s.inflight) < self.depth and s.launched < s.req.steps:
            try:
                tok = self.backend.launch(s.handle, s.launched, s.stream)
            except Exception as e:
                self._retire(s, FAILED, "step %d: %s" % (s.launched, e))
                return
            s.inflight.append(tok)
            s.launched += 1

    def _poll(self, s: Slot) -> bool:
        """Checks the request's finished steps in order; True if any."""
        progressed = False
        while s.state == ACTIVE and s.inflight and self.backend.ready(s.inflight[0]):
            tok = s.inflight.popleft()
            loss, g2 = self.backend.read(tok)
            s.loss, s.gnorm2 = loss, g2
            s.step += 1
            progressed = True
            if not (math.isfinite(loss) and math.isfinite(g2)):
                self._retire(s, FAILED, "non-finite loss or gradient at step %d" % (s.step - 1))
            elif s.step >= s.req.steps:
                self._retire(s, DONE)
        return progressed

    def tick(self) -> bool:
        """One pass of the scheduler: admit what has arrived and fits, keep
        every active request's own steps in flight, check the steps that
        finished and retire finished and failed requests.  Returns whether
        anything happened."""
        busy = False
        now = self.now()
        n_active = len(self.active())
        self._admit(now)
        busy |= len(self.active()) != n_active
        for s in self.active():
            before = s.launched
            self._launch(s)
            busy |= s.launched != before
        for s in self.active():
            busy |= self._poll(s)
        self.ticks += 1
        return busy

    def run(self, max_ticks: Optional[int] = None, idle_sleep: float = 2e-4,
            progress=None, every: float = 10.0):
        """Runs until every submitted request has ended.  Waits for future
        arrivals on the server clock.  `progress(server)` is called about
        every `every` seconds of the server clock."""
        n = 0
        t_next = self.now() + every
        while not self.idle() and (max_ticks is None or n < max_ticks):
            if not self.tick():
                time.sleep(idle_sleep)
            n += 1
            if progress is not None and self.now() >= t_next:
                progress(self)
                t_next = self.now() + every

    # ---- metrics
    def metrics(self) -> dict:
        done = [s for s in self.slots.values() if s.state == DONE]
        lat = [s.latency for s in done]
        wait = [s.t_admit - s.t_arrive for s in done]
        steps = sum(s.step for s in self.slots.values())
        span = (self.t_last_end - min(s.t_arrive for s in done)) if done else math.nan
        return {
            "done": len(done),
            "failed": sum(s.state == FAILED for s in self.slots.values()),
            "refused": sum(s.state == REFUSED for s in self.slots.values()),
            "cancelled": sum(s.state == CANCELLED for s in self.slots.values()),
            "steps": steps,
            "latency_s_p50": nearest_rank(lat, 50),
            "latency_s_p95": nearest_rank(lat, 95),
            "latency_s_p99": nearest_rank(lat, 99),
            "latency_s_max": max(lat) if lat else math.nan,
            "queue_wait_s_p50": nearest_rank(wait, 50),
            "queue_wait_s_p99": nearest_rank(wait, 99),
            "makespan_s": span,
            "steps_per_s": steps / span if done and span > 0 else math.nan,
            "reserved_bytes": self.reserved,
            "ticks": self.ticks,
        }
