"""Serving on the GPU: a mix of 2D and 3D requests stepped together gives
every request exactly the parameters it gets when run alone; a request
with a non-finite sinogram fails without disturbing the others."""
import numpy as np
import pytest

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
        srv = Server(budget_bytes=8 << 30)
        rid = srv.submit(r)
        srv.run()
        assert srv.status(rid).state == DONE, srv.status(rid).error
        alone.append(srv.status(rid).theta)
    bad_y = reqs[0].y.copy()
    bad_y.ravel()[7] = np.nan
    bad = Request(problem=reqs[0].problem, y=bad_y, steps=4)
    srv = Server(budget_bytes=8 << 30, n_streams=3)
    ids = [srv.submit(r) for r in reqs]
    bid = srv.submit(bad)
    srv.run()
    assert srv.status(bid).state == FAILED and "non-finite" in srv.status(bid).error
    for rid, ref in zip(ids, alone):
        s = srv.status(rid)
        assert s.state == DONE, s.error
        assert np.array_equal(s.theta, ref)
    m = srv.metrics()
    say("serving mix metrics", m)
    assert m["done"] == 3 and m["failed"] == 1 and m["reserved_bytes"] == 0
