"""GPU parity: each library call against the FP64 oracle on the same seeded
inputs (tolerances: FP32 projections 1e-5, FP32 gradients 1e-4, BF16
gradients 2e-2, all relative in the 2-norm over the whole output)."""
import math

import numpy as np
import pytest
import torch

from oracle import geometry as ogeo
from oracle import grid as ogrid
from oracle import inr as oinr
from oracle import joseph, loss as oloss, sampler as osampler, adam as oadam
from paper_2604_09884_amd import configs, synth
from tests.gpu_util import dev, host, rel, report, say

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng


def _ops():
    from paper_2604_09884_amd import ops
    return ops


def _problems():
    return [
        ("c1", configs.C1),
        ("par2d-ragged", configs.par2d_problem(37, 7, 53)),
        ("cone-small", configs.cone_problem(24, 5, 20).with_(n_v=18, dv=3.1 / 18)),
        ("cone-ragged", configs.cone_problem(19, 3, 70).with_(n_v=9, dv=3.1 / 9)),
        # detector rows 0.68 voxel apart along z: the adjoint's branch-free
        # two-rows-per-voxel walk
        ("cone-w2", configs.cone_problem(40, 5, 60)),
        # the same walk with 2.5 detector columns per voxel and axis-aligned
        # views (about four columns cover each voxel)
        ("cone-walk2", configs.cone_problem(32, 4, 83).with_(n_v=44, dv=3.1 / 44)),
        # views at 45 degree multiples: tiles whose columns change principal
        # axis take the direct-gather route
        ("cone-45deg", configs.cone_problem(26, 8, 36).with_(n_v=20, dv=3.1 / 20)),
        # detector pixels several voxels wide: footprints beyond the LDS
        # capacity take the direct-gather route
        ("cone-coarse", configs.cone_problem(80, 3, 12).with_(n_v=40, dv=3.1 / 40)),
        # detector pixels a small fraction of a voxel: adjoint footprints
        # beyond the LDS capacity read the residual in place
        ("cone-fine", configs.cone_problem(16, 3, 200).with_(n_v=120, dv=3.1 / 120)),
        ("fan-small", configs.fan2d_problem(32, 12, 45)),
        ("fan-ragged", configs.fan2d_problem(37, 7, 53)),
        ("fan-wide", configs.fan2d_problem(41, 9, 61, du=5.0 / 61)),
    ]


def test_cone_cases_cover_every_adjoint_kind():
    from paper_2604_09884_amd import lib as L
    ops = _ops()
    kinds = {}
    for name, p in _problems():
        if p.dim == 3:
            g = ops.Geometry(p)
            kinds[name] = g.adjoint_kind
            g.close()
    say("adjoint kinds", kinds)
    assert {L.INRCT_ADJ_DIRECT, L.INRCT_ADJ_WALK, L.INRCT_ADJ_WALK2} <= set(kinds.values())


@pytest.mark.parametrize("name,p", _problems(), ids=[n for n, _ in _problems()])
def test_project_and_backproject_match_oracle(name, p):
    ops = _ops()
    say("case", name)
    g = ops.Geometry(p)
    say(name, "adjoint kind", g.adjoint_kind)
    P = joseph.problem_matrix(p)
    u = RNG(1).standard_normal(p.n_grid)
    r = RNG(2).standard_normal(P.shape[0])
    z = host(ops.ct_project(g, dev(u)))
    v = host(ops.ct_backproject(g, dev(r)))
    ez, ev = rel(z, P @ u), rel(v, P.T @ r)
    say(name, "P rel", ez, "P^T rel", ev)
    report(name, "fp32", "P", ez, 1e-5)
    report(name, "fp32", "P^T", ev, 1e-5)
    assert ez <= 1e-5 and ev <= 1e-5
    # adjoint identity of the GPU pair, dot products in float64
    zz = host(ops.ct_project(g, dev(u)))
    lhs, rhs = float(zz.ravel() @ r), float(u @ v.ravel())
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(zz) * np.linalg.norm(r)
    # gather at an index list is the same arithmetic
    idx = np.sort(RNG(3).choice(p.n_grid, size=min(500, p.n_grid), replace=False))
    va = host(ops.ct_backproject_at(g, dev(r), dev(idx, torch.int32)))
    assert np.allclose(va, v.ravel()[idx], rtol=1e-6, atol=1e-6 * np.abs(v).max())


def test_residual_ls_and_fls():
    ops = _ops()
    p = configs.C1
    g = ops.Geometry(p)
    z = RNG(4).standard_normal(g.n_rays).astype(np.float32)
    y = RNG(5).standard_normal(g.n_rays).astype(np.float32)
    r, lo = ops.residual_loss(g, dev(z), dev(y), 0)
    rr = host(r)
    assert rel(rr, oloss.ls_residual(z, y)) <= 1e-7
    # L is reduced in float64 from the float32 residual the kernel formed:
    # equal to that sum up to float64 summation order, and to the exact loss
    # up to the float32 rounding of z - y
    assert abs(host(lo) - 0.5 * float(rr.ravel() @ rr.ravel())) <= 1e-12 * oloss.ls_loss(z, y)
    assert abs(host(lo) - oloss.ls_loss(z, y)) <= 1e-7 * oloss.ls_loss(z, y)
    zz, yy = z.reshape(g.proj_shape), y.reshape(g.proj_shape)
    r, lo = ops.residual_loss(g, dev(z), dev(y), 1)
    ref = oloss.fls_residual(zz, yy, p.du)
    assert rel(host(r), ref) <= 1e-5
    assert abs(host(lo) - oloss.fls_loss(zz, yy, p.du)) <= 1e-5 * abs(oloss.fls_loss(zz, yy, p.du))


# detector widths that reach every layout of the register-tiled ramp filter
# (four, two and one rows a workgroup; 7 and 9 outputs a thread) and, past
# 3328 bins, the direct filter
FLS_CASES = [
    ("par2d-725", configs.par2d_problem(512, 9, 725)),
    ("cone3d-768", configs.cone_problem(64, 2, 768)),
    ("par2d-1000", configs.par2d_problem(512, 5, 1000)),
    ("par2d-2001", configs.par2d_problem(1024, 3, 2001)),
    ("par2d-3400", configs.par2d_problem(1024, 2, 3400)),
]


@pytest.mark.parametrize("name,p", FLS_CASES, ids=[c[0] for c in FLS_CASES])
def test_fls_residual_detector_widths(name, p):
    ops = _ops()
    g = ops.Geometry(p)
    z = RNG(6).standard_normal(g.n_rays).astype(np.float32)
    y = RNG(7).standard_normal(g.n_rays).astype(np.float32)
    zz, yy = z.reshape(g.proj_shape), y.reshape(g.proj_shape)
    r, lo = ops.residual_loss(g, dev(z), dev(y), 1)
    ref = oloss.fls_residual(zz, yy, p.du)
    L_ref = oloss.fls_loss(zz, yy, p.du)
    e = rel(host(r), ref)
    say("FLS %s: rows %d x %d bins, r rel %.3e, loss rel %.3e"
        % (name, g.n_rays // p.n_u, p.n_u, e, abs(host(lo) - L_ref) / abs(L_ref)))
    report(name, "fp32", "FLS residual F(z - y)", e, 1e-5)
    assert e <= 1e-5
    assert abs(host(lo) - L_ref) <= 1e-5 * abs(L_ref)


ARCHS = [
    ("ffn2d-128", configs.C1.arch, configs.par2d_problem(45, 20, 67)),
    ("siren2d-256", configs.C2.arch, configs.par2d_problem(41, 20, 61)),
    ("ffn3d-256", configs.C4.arch, configs.cone_problem(13, 6, 20)),
    ("ffn2d-512", configs.C6.arch, configs.fan2d_problem(45, 20, 67)),
]


def _away_from_kinks(theta, B, arch, X, margin):
    """Rows of X whose pre-activations all lie farther than margin * rms
    from 0 (ReLU decisions there cannot flip between FP64 and the kernel's
    precision)."""
    if arch.kind != "ffn":
        return np.ones(X.shape[0], bool)
    _, _, pre = oinr.forward(theta, B, X, arch, keep=True)
    ok = np.ones(X.shape[0], bool)
    for z in pre:
        ok &= np.all(np.abs(z) > margin * np.sqrt(np.mean(z * z)), axis=1)
    return ok


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
@pytest.mark.parametrize("name,arch,prob", ARCHS, ids=[a[0] for a in ARCHS])
def test_eval_and_vjp_match_oracle(name, arch, prob, dtype):
    from oracle import step as ostep
    ops = _ops()
    say("case", name, dtype)
    dim, N = prob.dim, prob.N
    theta, B = synth.random_theta(arch, 7)
    fov = ogrid.fov_indices(dim, N)
    m = ops.Model(arch, dim, N, dtype, max_k=fov.size)
    th, Bd = dev(theta), dev(B.reshape(-1) if B.size else np.zeros(1))
    u = host(ops.inr_eval_grid(m, th, Bd))
    u_ref = oinr.eval_grid(theta, B, arch, dim, N, fov, ogrid.coords).ravel()
    tol = 1e-4 if dtype == "fp32" else 2e-2
    eu = rel(u, u_ref)
    say(name, dtype, "E rel", eu)
    report(name + " (INR only)", dtype, "E", eu, tol)
    assert eu <= tol
    assert np.all(u.ravel()[np.setdiff1d(np.arange(N ** dim), fov)] == 0)
    # Eq. (2) on a ragged subset with the cotangent of Algorithm 1:
    # v = P^T (P E f - y) from the oracle, y the closed-form data
    op = ostep.Problem(prob.with_(arch=arch))
    y = synth.sinogram(prob.with_(n_ellipses=4), noisy=False).ravel()
    v_alg = op.P.T @ (op.P @ op.E(theta, B) - y)
    k = max(1, (fov.size * 2) // 3 - 5)
    idx = np.sort(RNG(8).choice(fov, size=k, replace=False))
    scale = fov.size / k
    g = host(ops.inr_vjp_subsampled(m, th, Bd, dev(idx, torch.int32), dev(v_alg), scale))
    g_ref = oinr.vjp(theta, B, ogrid.coords(dim, N, idx), scale * v_alg[idx], arch)
    eg = rel(g, g_ref)
    say(name, dtype, "g rel (Algorithm-1 cotangent)", eg)
    report(name + " (INR only)", dtype, "g, Algorithm-1 cotangent", eg, tol)
    assert eg <= tol
    # compact v gives the same result
    g2 = host(ops.inr_vjp_subsampled(m, th, Bd, dev(idx, torch.int32), dev(v_alg[idx]), scale,
                                     v_compact=True))
    assert np.array_equal(g, g2)
    # point evaluation
    f = host(ops.inr_eval_points(m, th, Bd, dev(idx, torch.int32)))
    assert rel(f, u_ref[idx]) <= tol
    if dtype == "fp32":
        # random-sign cotangents on points away from every ReLU kink
        keep = _away_from_kinks(theta, B, arch, ogrid.coords(dim, N, fov), 2e-4)
        idx2 = fov[keep]
        vr = RNG(9).standard_normal(idx2.size)
        g = host(ops.inr_vjp_subsampled(m, th, Bd, dev(idx2, torch.int32), dev(vr), 2.0,
                                        v_compact=True))
        g_ref = oinr.vjp(theta, B, ogrid.coords(dim, N, idx2), 2.0 * vr, arch)
        say(name, dtype, "g rel (random cotangent, %d points)" % idx2.size, rel(g, g_ref))
        assert rel(g, g_ref) <= 1e-4


@pytest.mark.parametrize("n_N,k", [((2, 16), 1), ((2, 45), 700), ((3, 40), 20000)])
def test_sampler_matches_oracle(n_N, k):
    ops = _ops()
    dim, N = n_N
    m = ops.Model(configs.C1.arch if dim == 2 else configs.C4.arch, dim, N, "fp32", max_k=k)
    fov = ogrid.fov_indices(dim, N)
    for step in (0, 3):
        got = host(ops.sample(m, 4242, step, k)).astype(np.int64)
        ref = osampler.sample_indices(fov, k, 4242, step)
        assert np.array_equal(got, ref)


def test_adam_matches_oracle():
    ops = _ops()
    arch = configs.C1.arch
    m = ops.Model(arch, 2, 16, "fp32", max_k=10)
    p = m.n_params
    rng = RNG(21)
    th = rng.standard_normal(p)
    ms, vs = np.zeros(p), np.zeros(p)
    tt, mm, vv = dev(th), dev(ms), dev(vs)
    for t in range(1, 6):
        gg = rng.standard_normal(p)
        gn = ops.adam(m, tt, mm, vv, dev(gg), t, 1e-3)
        th, ms, vs = oadam.adam_update(th, ms, vs, gg.astype(np.float32).astype(np.float64), t, 1e-3)
        assert abs(host(gn) - float(gg.astype(np.float32).astype(np.float64) @ gg.astype(np.float32).astype(np.float64))) < 1e-9 * p
    assert np.abs(host(tt) - th).max() <= 1e-6 * max(1.0, np.abs(th).max())
