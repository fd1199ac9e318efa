"""Serving on the GPU: requests that arrive while others run are admitted
and overlap on the device; every request ends with exactly the parameters
it gets when run alone; a request with a non-finite sinogram fails without
disturbing the others; a mixed request follows the oracle's trajectory."""
import numpy as np
import pytest

from oracle import sampler as osampler
from oracle import step as ostep
from paper_2604_09884_amd import configs, synth
from paper_2604_09884_amd.serve import DONE, FAILED, Request, Server
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _mix():
    c1 = configs.C1.with_(steps=4)
    siren = configs.par2d_problem(64, 30, 91, arch=configs.C2.arch, k_frac=1 / 16,
                                  lr=1e-4, mlp_dtype="bf16", n_ellipses=6, seed_phantom=1101,
                                  seed_init=3101, seed_sampler=4101)
    cone = configs.cone_problem(24, 8, 40, arch=configs.C3.arch, k_frac=0.25, lr=1e-3,
                                mlp_dtype="bf16", n_ellipses=6, seed_phantom=1102,
                                seed_init=3102, seed_sampler=4102)
    out = []
    for p, steps in ((c1, 4), (siren, 3), (cone, 5)):
        y = synth.sinogram(p).astype(np.float32)
        out.append(Request(problem=p, y=y, steps=steps))
    return out


def test_mix_equals_alone_and_failures_are_isolated():
    reqs = _mix()
    alone = []
    for r in reqs:
        srv = Server(budget_bytes=8 << 30, n_slots=1)
        rid = srv.submit(r)
        srv.run()
        assert srv.status(rid).state == DONE, srv.status(rid).error
        alone.append(srv.status(rid).theta)
    bad_y = reqs[0].y.copy()
    bad_y.ravel()[7] = np.nan
    bad = Request(problem=reqs[0].problem, y=bad_y, steps=4)
    srv = Server(budget_bytes=8 << 30, n_slots=3)
    # staggered arrivals: the later requests arrive while the first ones run
    ids = [srv.submit(r, arrival=0.02 * i) for i, r in enumerate(reqs)]
    bid = srv.submit(bad, arrival=0.01)
    srv.run()
    assert srv.status(bid).state == FAILED and "non-finite" in srv.status(bid).error
    for rid, ref in zip(ids, alone):
        s = srv.status(rid)
        assert s.state == DONE, s.error
        assert np.array_equal(s.theta, ref)
        assert s.t_admit >= s.t_arrive and s.latency > 0
    m = srv.metrics()
    say("serving mix metrics", m)
    assert m["done"] == 3 and m["failed"] == 1 and m["reserved_bytes"] == 0


def test_mixed_request_follows_the_oracle():
    # the C1 request of the mix against the oracle's own four Algorithm-1 +
    # Adam steps: final-image MSE within 2%, parameters close
    reqs = _mix()
    srv = Server(budget_bytes=8 << 30, n_slots=3)
    ids = [srv.submit(r) for r in reqs]
    srv.run()
    s = srv.status(ids[0])
    assert s.state == DONE, s.error
    p = reqs[0].problem
    prob = ostep.Problem(p)
    theta0, B = synth.init_inr(p.arch, p.seed_init)
    y = reqs[0].y.astype(np.float64)
    th, mm, vv = theta0.copy(), np.zeros_like(theta0), np.zeros_like(theta0)
    for t in range(p.steps):
        idx = osampler.sample_indices(prob.fov, p.k(prob.n), p.seed_sampler, t)
        th, mm, vv, _, _ = ostep.grad_step(prob, th, B, mm, vv, t + 1, y, idx, p.lr)
    truth = synth.raster(synth.phantom(p), 2, p.N)
    mse_ref = ostep.mse(prob.E(th, B), truth, prob.fov)
    mse_gpu = ostep.mse(prob.E(s.theta.astype(np.float64), B), truth, prob.fov)
    dth = np.linalg.norm(s.theta - th) / np.linalg.norm(th - theta0)
    say("mixed C1 request after %d steps: MSE %.6g (oracle %.6g), |dtheta| rel to the "
        "oracle's update %.3e" % (p.steps, mse_gpu, mse_ref, dth))
    assert abs(mse_gpu - mse_ref) <= 0.02 * mse_ref
    assert dth <= 1e-2
