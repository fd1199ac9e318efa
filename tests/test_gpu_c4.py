"""GPU parity at the full 501^3, 20-view, 768^2 cone-beam size, on outputs
the oracle can compute one by one: sampled rays of P, sampled voxels of
P^T, sampled points of E, and the whole index set of the sampler."""
import numpy as np
import pytest
import torch

from oracle import geometry as ogeo
from oracle import grid as ogrid
from oracle import inr as oinr
from oracle import joseph
from oracle import sampler as osampler
from paper_2604_09884_amd import configs, synth
from tests.gpu_util import dev, host, rel, report, say

pytestmark = pytest.mark.gpu

P4 = configs.C4
RNG = np.random.default_rng


def _smooth_volume(N):
    c = ogrid.centres(N)
    gx = np.exp(-((c - 0.1) ** 2) / 0.18)
    gy = np.cos(2.5 * c) + 0.3 * c
    gz = np.exp(-((c + 0.2) ** 2) / 0.3)
    return (gz[:, None, None] * gy[None, :, None] * gx[None, None, :]).astype(np.float32)


@pytest.fixture(scope="module")
def geom():
    from paper_2604_09884_amd import ops
    return ops.Geometry(P4)


def test_c4_projection_sampled_rays(geom):
    from paper_2604_09884_amd import ops
    N = P4.N
    u = _smooth_volume(N)
    z = host(ops.ct_project(geom, dev(u.ravel())))
    rng = RNG(11)
    views = rng.choice(P4.n_views, size=6, replace=False)
    got, ref = [], []
    for j in views:
        rows = np.sort(rng.choice(P4.n_v, size=3, replace=False))
        cols = np.sort(rng.choice(P4.n_u, size=12, replace=False))
        p0, d = ogeo.cone3d_rays(P4.n_views, P4.n_u, P4.n_v, P4.du, P4.dv, P4.dso, P4.dod,
                                 views=[j], rows=rows, cols=cols)
        A = joseph.system_matrix(N, 3, p0, d)
        ref.append(A @ u.ravel().astype(np.float64))
        got.append(z[j][np.ix_(rows, cols)].ravel())
    e = rel(np.concatenate(got), np.concatenate(ref))
    say("C4 sampled-ray P rel", e)
    report("cone3d-501 (C4)", "fp32", "P, sampled rays", e, 1e-5)
    assert e <= 1e-5


def _window_adjoint(vox, r3, N):
    """(P^T r) at one voxel from every ray of a window around the voxel's
    projection in each view; the window border must carry zero weight."""
    x, y, zc = ogrid.coords(3, N, [vox])[0]
    tot = 0.0
    for j in range(P4.n_views):
        ph = j * (P4.view_span / P4.n_views)
        S = np.array([P4.dso * np.cos(ph), P4.dso * np.sin(ph), 0.0])
        C = -P4.dod * np.array([np.cos(ph), np.sin(ph), 0.0])
        eu = np.array([-np.sin(ph), np.cos(ph), 0.0])
        X = np.array([x, y, zc])
        n = C - S
        t = np.dot(n, n) / np.dot(X - S, n)
        Q = S + t * (X - S)
        ua = np.dot(Q - C, eu) / P4.du + (P4.n_u - 1) / 2
        vb = Q[2] / P4.dv + (P4.n_v - 1) / 2
        c_lo, c_hi = int(np.floor(ua)) - 5, int(np.floor(ua)) + 6
        r_lo, r_hi = int(np.floor(vb)) - 5, int(np.floor(vb)) + 6
        cols = np.arange(max(c_lo, 0), min(c_hi, P4.n_u - 1) + 1)
        rows = np.arange(max(r_lo, 0), min(r_hi, P4.n_v - 1) + 1)
        if cols.size == 0 or rows.size == 0:
            continue
        p0, d = ogeo.cone3d_rays(P4.n_views, P4.n_u, P4.n_v, P4.du, P4.dv, P4.dso, P4.dod,
                                 views=[j], rows=rows, cols=cols)
        w = joseph.voxel_weights(N, 3, p0, d, vox).reshape(rows.size, cols.size)
        # window edges that are not the detector edge carry no weight
        if r_lo >= 0:
            assert np.all(w[0, :] == 0)
        if r_hi <= P4.n_v - 1:
            assert np.all(w[-1, :] == 0)
        if c_lo >= 0:
            assert np.all(w[:, 0] == 0)
        if c_hi <= P4.n_u - 1:
            assert np.all(w[:, -1] == 0)
        tot += float(np.sum(w * r3[j][np.ix_(rows, cols)]))
    return tot


def test_c4_backprojection_sampled_voxels(geom):
    from paper_2604_09884_amd import lib as L, ops
    # the benchmark geometry takes the branch-free walk
    assert geom.adjoint_kind == L.INRCT_ADJ_WALK2
    N = P4.N
    r = RNG(12).standard_normal(geom.n_rays).astype(np.float32)
    v = host(ops.ct_backproject(geom, dev(r))).ravel()
    r3 = r.reshape(geom.proj_shape).astype(np.float64)
    fov = ogrid.fov_indices(2, N)
    rng = RNG(13)
    vox = fov[rng.choice(fov.size, 40)] + rng.integers(0, N, 40) * N * N
    vox = np.concatenate([vox, [0, N * N * N - 1, N // 2 * (N * N + N + 1)]])
    ref = np.array([_window_adjoint(int(q), r3, N) for q in vox])
    e = rel(v[vox], ref)
    say("C4 sampled-voxel P^T rel", e)
    report("cone3d-501 (C4)", "fp32", "P^T, sampled voxels", e, 1e-5)
    assert e <= 1e-5
    va = host(ops.ct_backproject_at(geom, dev(r), dev(vox, torch.int32)))
    assert np.allclose(va, v[vox], rtol=1e-6, atol=1e-6 * np.abs(v).max())


def test_c4_adjoint_identity(geom):
    from paper_2604_09884_amd import ops
    u = RNG(14).standard_normal(geom.grid_shape[0] ** 3).astype(np.float32)
    r = RNG(15).standard_normal(geom.n_rays).astype(np.float32)
    z = host(ops.ct_project(geom, dev(u))).ravel()
    v = host(ops.ct_backproject(geom, dev(r))).ravel()
    lhs, rhs = float(z @ r), float(u.astype(np.float64) @ v)
    say("C4 <Pu,r> - <u,P^T r> relative", abs(lhs - rhs) / (np.linalg.norm(z) * np.linalg.norm(r)))
    report("cone3d-501 (C4)", "fp32", "adjoint identity <Pu,r> - <u,P^T r>", abs(lhs - rhs) / (np.linalg.norm(z) * np.linalg.norm(r)), 1e-5)
    assert abs(lhs - rhs) <= 1e-6 * np.linalg.norm(z) * np.linalg.norm(r)


def test_c4_grid_evaluation_sampled_points():
    from paper_2604_09884_amd import ops
    arch = P4.arch
    theta, B = synth.init_inr(arch, P4.seed_init)
    m = ops.Model(arch, 3, P4.N, "bf16", max_k=1000)
    u = host(ops.inr_eval_grid(m, dev(theta), dev(B.ravel()))).ravel()
    N = P4.N
    fov2 = ogrid.fov_indices(2, N)
    rng = RNG(16)
    pts = fov2[rng.choice(fov2.size, 3000)] + rng.integers(0, N, 3000) * N * N
    pts = np.unique(np.concatenate([pts, [fov2[0], fov2[-1] + (N - 1) * N * N]]))
    ref = oinr.forward(theta, B, ogrid.coords(3, N, pts), arch)
    e = rel(u[pts], ref)
    say("C4 E (bf16) sampled rel", e)
    report("cone3d-501 (C4)", "bf16", "E, sampled points", e, 2e-2)
    assert e <= 2e-2
    # outside the FOV the grid is zero
    outside = np.array([0, N - 1, N * N - 1, N * N * (N - 1)])
    assert np.all(u[outside] == 0)


def test_c4_sampler_full_index_set():
    from paper_2604_09884_amd import ops
    N = P4.N
    n = P4.n_fov()
    k = P4.k(n)
    m = ops.Model(P4.arch, 3, N, "bf16", max_k=k)
    got = host(ops.sample(m, P4.seed_sampler, 7, k)).astype(np.int64)
    ranks = osampler.sample_ranks_np(n, k, P4.seed_sampler, 7)
    # rank -> grid index through the FOV order of each z slice
    fov2 = ogrid.fov_indices(2, N)
    ref = (ranks // fov2.size) * N * N + fov2[ranks % fov2.size]
    assert np.array_equal(got, ref)
