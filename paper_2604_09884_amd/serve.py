"""Serving: many CT reconstructions stepped together on one GPU.

Each request is one reconstruction problem: a geometry, its sinogram y, an
INR architecture and optimiser settings.  Its parameters, Adam state, data
and all scratch stay resident on the device from admission to retirement.
A scheduler tick runs one gradient step (Algorithm 1 followed by Adam) of
every active request.  Steps of different requests go to a small pool of
HIP streams, so short kernels of one request overlap long ones of another.

Per-request results do not depend on the mix: each request owns its
buffers, the step kernels use no atomics and reduce in a fixed order, and
requests share nothing but the device.

Admission is by device memory: a request is admitted when its reservation
fits the remaining budget, in arrival order (a request that can never fit
is refused).  A request whose loss or gradient norm turns non-finite, or
whose launch raises, is retired as failed and its memory released; the
others keep running.  Requests can be cancelled between ticks.

The scheduler is host logic over a backend object.  `HipBackend` drives
the C ABI through `ops` (there is no other product backend; tests supply
their own stand-in to exercise the scheduling logic on the CPU).
"""
from __future__ import annotations

import dataclasses
import itertools
import math
import time
from typing import Any, Dict, List, Optional

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
    reserved: int = 0
    step: int = 0
    loss: float = math.nan
    gnorm2: float = math.nan
    error: str = ""
    t_submit: float = 0.0
    t_admit: float = 0.0
    t_end: float = 0.0
    theta: Any = None  # final parameters (host copy) once done


def reservation_bytes(p: Problem, mlp_dtype: Optional[str] = None) -> int:
    """Device bytes a request holds while resident (an upper estimate of the
    library's allocations for this problem)."""
    dtype = mlp_dtype or p.mlp_dtype
    n_grid = p.N ** p.dim
    pad = ((p.N + 4) / p.N) ** p.dim
    vol = 4 * n_grid * (2 + (2 * pad if p.geometry == "cone3d" else 0))  # u, v, padded copies
    rays = 4 * p.n_rays * 3                                               # y, r, step-scaled r
    params = p.arch.n_params
    opt = 4 * params * 6                                                  # theta, m, v, g, packs
    k = p.k(p.n_fov())
    P = min(262144, -(-k // 256) * 256)
    W, L = p.arch.width, p.arch.depth
    k1 = p.arch.enc_dim
    es = 2 if dtype == "bf16" else 4
    vjp = P * (k1 + 2 * L * W + 1) * es + P * 64                          # activations, deltas, masks
    ntiles = -(-k1 // 256) + L * -(-W // 256)                             # dW tiles
    kslice = min(2048, max(512, -(-(-(-P // -(-256 // ntiles))) // 256) * 256))
    part = -(-P // kslice) * ntiles * (256 * 257) * 4                      # dW partials
    frag = params * 2 * 4 * 2                                             # fragment streams
    flags = p.n_fov() + 4 * k
    if p.arch.kind == "hash":  # point rows, sorted contributions, dW slice partials
        R = k1 + 2 * L * W + 1
        nc = k * p.arch.hash_levels * (1 << p.dim)
        n_mlp = params - p.arch.n_table
        vjp = 4 * k * R + 24 * nc + 8 * nc
        part = 4 * -(-k // 256) * n_mlp
        frag = 0
    return int(1.1 * (vol + rays + opt + vjp + part + frag + flags)) + (8 << 20)


class HipBackend:
    """Creates a request's device state through `ops` and steps it on a
    given stream."""

    def __init__(self, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)

    def reservation(self, req: Request) -> int:
        return reservation_bytes(req.problem, req.mlp_dtype)

    def create(self, req: Request):
        from . import lib as L
        from . import ops, synth
        torch = self.torch
        p = req.problem
        dtype = req.mlp_dtype or p.mlp_dtype
        if req.theta0 is None:
            theta, B = synth.init_inr(p.arch, p.seed_init)
        else:
            theta, B = req.theta0, req.B
        th = torch.as_tensor(np.asarray(theta, dtype=np.float32) if not torch.is_tensor(theta)
                             else theta, dtype=torch.float32, device=self.device).clone()
        Bv = np.zeros(1, np.float32) if B is None or np.size(B) == 0 else np.asarray(B).ravel()
        Bd = torch.as_tensor(Bv, dtype=torch.float32, device=self.device)
        yd = torch.as_tensor(np.asarray(req.y, dtype=np.float32).ravel() if not torch.is_tensor(req.y)
                             else req.y.reshape(-1), dtype=torch.float32, device=self.device)
        model = ops.Model(p.arch, p.dim, p.N, dtype, max_k=p.k())
        geom = ops.Geometry(p)
        k = p.k(model.n_fov)
        v_mode = L.INRCT_V_FULL if req.v_mode == "full" else L.INRCT_V_AT_I
        st = ops.GradStepper(model, geom, th, Bd, yd, k, p.lr, seed=p.seed_sampler, v_mode=v_mode)
        return {"stepper": st, "model": model, "geom": geom}

    def step(self, h, t: int, stream):
        with self.torch.cuda.stream(stream):
            h["stepper"].step(t)

    def streams(self, n: int):
        return [self.torch.cuda.Stream(device=self.device) for _ in range(n)]

    def sync(self, streams):
        for s in streams:
            s.synchronize()

    def read(self, h):
        st = h["stepper"]
        return float(st.loss), float(st.gnorm2)

    def theta(self, h):
        return h["stepper"].theta.detach().cpu().numpy()

    def release(self, h):
        h["stepper"].close()
        h.clear()


class Server:
    """Continuous batching of gradient steps over resident requests."""

    def __init__(self, backend=None, budget_bytes: Optional[int] = None, n_streams: int = 4):
        self.backend = backend if backend is not None else HipBackend()
        if budget_bytes is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(free * 0.8)
        self.budget = int(budget_bytes)
        self.reserved = 0
        self.slots: Dict[int, Slot] = {}
        self.queue: List[int] = []
        self._ids = itertools.count()
        self.streams = self.backend.streams(max(1, n_streams))
        self.tick_ms: List[float] = []
        self.ticks = 0

    # ---- requests
    def submit(self, req: Request) -> int:
        rid = next(self._ids)
        s = Slot(rid, req, t_submit=time.perf_counter())
        s.reserved = int(self.backend.reservation(req))
        self.slots[rid] = s
        if s.reserved > self.budget:
            s.state, s.error = REFUSED, "reservation %d B exceeds the budget %d B" % (
                s.reserved, self.budget)
            s.t_end = time.perf_counter()
        else:
            self.queue.append(rid)
        return rid

    def cancel(self, rid: int):
        s = self.slots[rid]
        if s.state == QUEUED:
            self.queue.remove(rid)
            s.state, s.t_end = CANCELLED, time.perf_counter()
        elif s.state == ACTIVE:
            self._retire(s, CANCELLED)

    def status(self, rid: int) -> Slot:
        return self.slots[rid]

    def active(self) -> List[Slot]:
        return [s for s in self.slots.values() if s.state == ACTIVE]

    def idle(self) -> bool:
        return not self.queue and not self.active()

    # ---- scheduling
    def _admit(self):
        while self.queue:
            s = self.slots[self.queue[0]]
            if self.reserved + s.reserved > self.budget:
                break  # arrival order: later requests wait behind this one
            self.queue.pop(0)
            try:
                s.handle = self.backend.create(s.req)
            except Exception as e:  # creation failed: nothing stays reserved
                s.state, s.error, s.t_end = FAILED, "create: %s" % e, time.perf_counter()
                continue
            self.reserved += s.reserved
            s.state, s.t_admit = ACTIVE, time.perf_counter()

    def _retire(self, s: Slot, state: str, error: str = ""):
        try:
            self.backend.release(s.handle)
        finally:
            s.handle = None
            self.reserved -= s.reserved
            s.state, s.error, s.t_end = state, error, time.perf_counter()

    def tick(self):
        """Admit what fits, run one step of every active request, check the
        results, retire finished and failed requests."""
        t0 = time.perf_counter()
        self._admit()
        act = self.active()
        launched = []
        for i, s in enumerate(act):
            try:
                self.backend.step(s.handle, s.step, self.streams[i % len(self.streams)])
                launched.append(s)
            except Exception as e:
                self._retire(s, FAILED, "step %d: %s" % (s.step, e))
        self.backend.sync(self.streams)
        for s in launched:
            loss, g2 = self.backend.read(s.handle)
            s.loss, s.gnorm2 = loss, g2
            s.step += 1
            if not (math.isfinite(loss) and math.isfinite(g2)):
                self._retire(s, FAILED, "non-finite loss or gradient at step %d" % (s.step - 1))
            elif s.step >= s.req.steps:
                s.theta = self.backend.theta(s.handle)
                self._retire(s, DONE)
        self.ticks += 1
        if launched:
            self.tick_ms.append((time.perf_counter() - t0) * 1e3)

    def run(self, max_ticks: Optional[int] = None):
        n = 0
        while not self.idle() and (max_ticks is None or n < max_ticks):
            self.tick()
            n += 1

    # ---- metrics
    def metrics(self) -> dict:
        t = np.asarray(self.tick_ms) if self.tick_ms else np.zeros(1)
        done = [s for s in self.slots.values() if s.state == DONE]
        return {
            "ticks": self.ticks,
            "tick_ms_p50": float(np.percentile(t, 50)),
            "tick_ms_p99": float(np.percentile(t, 99)),
            "done": len(done),
            "failed": sum(s.state == FAILED for s in self.slots.values()),
            "refused": sum(s.state == REFUSED for s in self.slots.values()),
            "cancelled": sum(s.state == CANCELLED for s in self.slots.values()),
            "steps": sum(s.step for s in self.slots.values()),
            "reserved_bytes": self.reserved,
        }
