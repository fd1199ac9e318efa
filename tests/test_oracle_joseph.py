"""Pins for the oracle projector P and its transpose (CPU only).

Each check is independent of the oracle's own construction: closed-form
line integrals, exact special cases, a symmetry of the geometry, and a
second, slice-restricted evaluation of the same matrix entries."""
import math

import numpy as np
import pytest

from oracle import geometry, grid, joseph
from paper_2604_09884_amd import configs, synth


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def _small_cone(N=12, V=5, det=10):
    return geometry.cone3d_rays(V, det, det, 3.1 / det, 3.1 / det,
                                configs.CONE_DSO, configs.CONE_DOD)


def test_adjoint_identity_2d_3d():
    for N, dim, (p0, d) in [(16, 2, geometry.par2d_rays(12, 25, 1 / 8)),
                            (10, 3, _small_cone(10))]:
        A = joseph.system_matrix(N, dim, p0, d)
        u = _rand(N ** dim, 1)
        r = _rand(p0.shape[0], 2)
        Pu = joseph.project(u, N, dim, p0, d)
        PTr = joseph.backproject(r, N, dim, p0, d).ravel()
        lhs, rhs = Pu @ r, u @ PTr
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Pu) * np.linalg.norm(r)
        # dense transpose from unit vectors
        D = np.stack([joseph.project(e, N, dim, p0, d)
                      for e in np.eye(N ** dim)[:40]], axis=1)
        DT = np.stack([joseph.backproject(e, N, dim, p0, d).ravel()
                       for e in np.eye(p0.shape[0])], axis=0)[:, :40]
        assert np.abs(D - DT).max() <= 1e-15 * max(1.0, np.abs(D).max())


def test_view0_closed_form_column_sums():
    # theta = 0, N even, K odd, du = h: every ray lies halfway between two
    # pixel columns, so z_k = h (colsum[k-29]/2 + colsum[k-28]/2) for C1.
    p = configs.C1
    N, K = p.N, p.n_u
    u = _rand((N, N), 3)
    p0, d = geometry.par2d_rays(p.n_views, K, p.du, views=[0])
    z = joseph.project(u, N, 2, p0, d)
    cs = u.sum(axis=0)
    off = (K - N) // 2 + 1          # 29
    ref = np.zeros(K)
    for k in range(K):
        for i, w in ((k - off, 0.5), (k - off + 1, 0.5)):
            if 0 <= i < N:
                ref[k] += p.h * w * cs[i]
    assert np.abs(z - ref).max() <= 1e-13 * np.abs(ref).max()
    # theta = 90 deg (view 30): same with row sums (x-principal ray)
    p0, d = geometry.par2d_rays(p.n_views, K, p.du, views=[30])
    z = joseph.project(u, N, 2, p0, d)
    rs = u.sum(axis=1)
    ref = np.zeros(K)
    for k in range(K):
        for i in (k - off, k - off + 1):
            if 0 <= i < N:
                ref[k] += p.h * 0.5 * rs[i]
    assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()


def test_constant_image_is_path_length():
    # u = 1 on the whole grid: a ray whose slice crossings all fall inside the
    # grid integrates to N * h / |cos| = 2 / |cos| (its length in the square).
    N = 64
    u = np.ones((N, N))
    th = np.deg2rad(np.array([0.0, 7.0, 21.0, 40.0, 100.0, 155.0]))
    p0 = np.zeros((th.size, 2)) + 0.01 * np.stack([np.cos(th), np.sin(th)], 1)
    d = np.stack([-np.sin(th), np.cos(th)], 1)
    z = joseph.project(u, N, 2, p0, d)
    lead = np.maximum(np.abs(d[:, 0]), np.abs(d[:, 1]))
    assert np.allclose(z, 2.0 / lead, rtol=1e-13)


def test_gaussian_blob_2d_second_order():
    sig, cen = 0.15, np.array([0.1, -0.05])
    errs = []
    for N in (64, 128, 256):
        c = grid.centres(N)
        Y, X = np.meshgrid(c, c, indexing="ij")
        u = np.exp(-((X - cen[0]) ** 2 + (Y - cen[1]) ** 2) / (2 * sig ** 2))
        p0, d = geometry.par2d_rays(7, 2 * N + 1, 1.0 / N)
        z = joseph.project(u, N, 2, p0, d)
        dn = d / np.linalg.norm(d, axis=1)[:, None]
        rel = cen[None, :] - p0
        rho = np.abs(rel[:, 0] * dn[:, 1] - rel[:, 1] * dn[:, 0])
        ref = math.sqrt(2 * math.pi) * sig * np.exp(-rho ** 2 / (2 * sig ** 2))
        errs.append(np.linalg.norm(z - ref) / np.linalg.norm(ref))
    assert errs[1] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_gaussian_blob_cone_second_order():
    sig, cen = 0.2, np.array([0.1, -0.05, 0.08])
    errs = []
    for N in (32, 64):
        c = grid.centres(N)
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        u = np.exp(-((X - cen[0]) ** 2 + (Y - cen[1]) ** 2 + (Z - cen[2]) ** 2)
                   / (2 * sig ** 2))
        p0, d = geometry.cone3d_rays(5, 24, 24, 3.1 / 24, 3.1 / 24,
                                     configs.CONE_DSO, configs.CONE_DOD)
        z = joseph.project(u, N, 3, p0, d)
        dn = d / np.linalg.norm(d, axis=1)[:, None]
        rho = np.linalg.norm(np.cross(cen[None, :] - p0, dn), axis=1)
        ref = math.sqrt(2 * math.pi) * sig * np.exp(-rho ** 2 / (2 * sig ** 2))
        errs.append(np.linalg.norm(z - ref) / np.linalg.norm(ref))
    assert errs[1] < 4e-3
    assert errs[0] / errs[1] > 3.5


def test_disc_raster_converges_to_chords():
    # rasterised ellipses vs exact chord integrals: error falls with N
    ph = synth.random_ellipses(4, seed=5)
    errs = []
    for N in (64, 128, 256):
        u = synth.raster(ph, 2, N)
        p0, d = geometry.par2d_rays(9, 2 * N + 1, 1.0 / N)
        z = joseph.project(u, N, 2, p0, d)
        ref = synth.chord_integrals(ph, 2, p0, d)
        errs.append(np.linalg.norm(z - ref) / np.linalg.norm(ref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.02


def test_rotation_by_90_degrees_is_a_view_shift():
    # rotating the image by +90 deg maps ray (theta, s) to (theta + pi/2, s);
    # C1 has 60 views over 180 deg, so that is a shift of 30 views.  The
    # 45 and 135 degree views are principal-axis ties and are excluded.
    p = configs.C1
    N, K, V = p.N, p.n_u, p.n_views
    u = _rand((N, N), 4)
    u_rot = np.empty_like(u)
    for iy in range(N):
        for ix in range(N):
            u_rot[iy, ix] = u[N - 1 - ix, iy]
    p0, d = geometry.par2d_rays(V, K, p.du)
    z = joseph.project(u, N, 2, p0, d).reshape(V, K)
    zr = joseph.project(u_rot, N, 2, p0, d).reshape(V, K)
    for j in range(V // 2):
        if j in (15, 45 - 30):
            continue
        assert np.allclose(zr[j + V // 2], z[j], atol=1e-12 * np.abs(z).max())


def test_voxel_weights_equal_matrix_entries():
    for N, dim, (p0, d) in [(16, 2, geometry.par2d_rays(12, 25, 1 / 8)),
                            (12, 3, _small_cone(12, V=6, det=12))]:
        A = joseph.system_matrix(N, dim, p0, d).tocsc()
        rng = np.random.default_rng(8)
        for vox in rng.choice(N ** dim, size=25, replace=False):
            col = A[:, vox].toarray().ravel()
            w = joseph.voxel_weights(N, dim, p0, d, vox)
            assert np.abs(col - w).max() <= 1e-14


def test_principal_axis_tie_rule():
    # exact 45 and 135 degree rays are y-principal (|d_y| >= (1-tau)|d_x|)
    th = np.array([np.pi / 4, 3 * np.pi / 4, np.pi / 4 + 1e-6])
    d = np.stack([-np.sin(th), np.cos(th)], 1)
    ypr = joseph.y_principal(d)
    assert ypr[0] and ypr[1] and not ypr[2]


# ------------------------------------------------------------ 2D fan beam
def _fan(N=64, V=12, K=None, span=2 * np.pi):
    K = K or N
    return geometry.fan2d_rays(V, K, configs.CONE_DET_WIDTH / K, configs.CONE_DSO,
                               configs.CONE_DOD, span)


def test_fan_rays_geometry():
    # every ray starts at the source (distance D_so from the centre), ends on
    # the detector line (distance D_od on the far side), bins are du apart
    # along the detector, and the middle bin of an odd detector passes
    # through the centre; the generator behind the data agrees.
    V, K = 7, 33
    du = 3.1 / K
    p0, d = geometry.fan2d_rays(V, K, du, 31.25, 15.625)
    assert np.allclose(np.linalg.norm(p0, axis=1), 31.25, rtol=1e-14)
    ph = np.repeat(np.arange(V) * (2 * np.pi / V), K)
    n = np.stack([np.cos(ph), np.sin(ph)], 1)
    Q = p0 + d
    assert np.allclose(np.einsum("ij,ij->i", Q, n), -15.625, atol=1e-12)
    gaps = np.linalg.norm(np.diff(Q.reshape(V, K, 2), axis=1), axis=2)
    assert np.allclose(gaps, du, rtol=1e-10)
    mid = p0.reshape(V, K, 2)[:, K // 2], d.reshape(V, K, 2)[:, K // 2]
    cross = mid[0][:, 0] * mid[1][:, 1] - mid[0][:, 1] * mid[1][:, 0]
    assert np.abs(cross).max() <= 1e-12 * 31.25 * 46.875
    sp0, sd = synth.rays_fan2d(V, K, du, 31.25, 15.625)
    assert np.allclose(sp0, p0, atol=1e-13) and np.allclose(sd, d, atol=1e-13)


def test_fan_constant_image_is_chord_length():
    # u = 1: a ray whose crossings of the first and last slice planes both
    # fall between the outermost pixel centres of the other axis sees weight
    # 1 at every slice, so it integrates to its chord through the square,
    # 2 |d| / |d_axis|.  Checked for every such ray of the fan.
    # (a detector 5 units wide, so that outer bins miss the square)
    N = 64
    p0, d = geometry.fan2d_rays(16, 101, 5.0 / 101, configs.CONE_DSO, configs.CONE_DOD)
    z = joseph.project(np.ones(N * N), N, 2, p0, d)
    ax = np.where(np.abs(d[:, 1]) >= np.abs(d[:, 0]), 1, 0)
    rows = np.arange(p0.shape[0])
    da, pa = d[rows, ax], p0[rows, ax]
    do_, po = d[rows, 1 - ax], p0[rows, 1 - ax]
    lim = 1.0 - 1.0 / N
    inside = np.ones(p0.shape[0], bool)
    for q in (-1.0 + 1.0 / N, 1.0 - 1.0 / N):
        t = (q - pa) / da
        inside &= np.abs(po + t * do_) <= lim
    assert inside.sum() > 200
    chord = 2.0 * np.linalg.norm(d, axis=1) / np.abs(da)
    assert np.allclose(z[inside], chord[inside], rtol=1e-12)
    # rays that miss the square see nothing
    miss = np.ones(p0.shape[0], bool)
    for q in (-1.0, 1.0):
        t = (q - pa) / da
        miss &= np.abs(po + t * do_) > 1.0 + 2.0 / N
    assert miss.sum() > 0 and np.all(z[miss] == 0)


def test_fan_gaussian_blob_second_order():
    sig, cen = 0.15, np.array([0.1, -0.05])
    errs = []
    for N in (64, 128, 256):
        c = grid.centres(N)
        Y, X = np.meshgrid(c, c, indexing="ij")
        u = np.exp(-((X - cen[0]) ** 2 + (Y - cen[1]) ** 2) / (2 * sig ** 2))
        p0, d = _fan(N, V=9, K=129)
        z = joseph.project(u, N, 2, p0, d)
        dn = d / np.linalg.norm(d, axis=1)[:, None]
        rel = cen[None, :] - p0
        rho = np.abs(rel[:, 0] * dn[:, 1] - rel[:, 1] * dn[:, 0])
        ref = math.sqrt(2 * math.pi) * sig * np.exp(-rho ** 2 / (2 * sig ** 2))
        errs.append(np.linalg.norm(z - ref) / np.linalg.norm(ref))
    assert errs[1] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_fan_rotation_by_90_degrees_is_a_view_shift():
    # 180 views over 360 deg: rotating the image by +90 deg maps view j's
    # rays onto view j + 45's.  Rays within 1e-6 of a principal-axis tie
    # are excluded (rotation swaps the axes there).
    N, V, K = 48, 180, 64
    u = _rand((N, N), 6)
    u_rot = np.empty_like(u)
    for iy in range(N):
        for ix in range(N):
            u_rot[iy, ix] = u[N - 1 - ix, iy]
    views = np.arange(0, 180, 7)
    p0, d = _fan(N, V=V, K=K)
    sel = (views[:, None] * K + np.arange(K)[None, :]).ravel()
    sel2 = (((views[:, None] + 45) % V) * K + np.arange(K)[None, :]).ravel()
    z = joseph.project(u, N, 2, p0[sel], d[sel])
    zr = joseph.project(u_rot, N, 2, p0[sel2], d[sel2])
    dd = d[sel]
    ok = np.abs(np.abs(dd[:, 0]) - np.abs(dd[:, 1])) > 1e-6 * np.linalg.norm(dd, axis=1)
    assert ok.sum() > 0.9 * ok.size
    assert np.allclose(zr[ok], z[ok], atol=1e-11 * np.abs(z).max())


def test_fan_adjoint_and_voxel_weights():
    N = 20
    p0, d = _fan(N, V=9, K=29)
    A = joseph.system_matrix(N, 2, p0, d)
    u, r = _rand(N * N, 7), _rand(p0.shape[0], 8)
    assert abs((A @ u) @ r - u @ (A.T @ r)) <= 1e-12 * np.linalg.norm(A @ u) * np.linalg.norm(r)
    Ac = A.tocsc()
    for vox in np.random.default_rng(9).choice(N * N, size=25, replace=False):
        col = Ac[:, vox].toarray().ravel()
        assert np.abs(col - joseph.voxel_weights(N, 2, p0, d, vox)).max() <= 1e-14


def test_fan_large_distance_approaches_parallel():
    # with the source and detector 1e7 away and the detector pitch scaled by
    # the magnification 2, the fan view at angle phi has rays within ~1e-7
    # rad of the parallel view at phi + pi/2 (same direction -(cos, sin) and
    # detector axis (-sin, cos)), bin for bin.
    N, V, K = 32, 6, 45
    u = _rand(N * N, 10)
    du = 2.0 / N
    pf, df = geometry.fan2d_rays(V, K, 2 * du, 1e7, 1e7, span=np.pi)
    zf = joseph.project(u, N, 2, pf, df).reshape(V, K)
    for j in range(V):
        th = j * np.pi / V + np.pi / 2
        pq, dq = geometry.par2d_rays(1, K, du, span=th, views=[1])
        zq = joseph.project(u, N, 2, pq, dq)
        assert np.abs(zq - zf[j]).max() <= 1e-5 * np.abs(zq).max()


# ------------------------------------------------------------ 3D cone beam
def test_cone_rays_geometry():
    # Every ray starts at the source, on the circle of radius D_so in the
    # plane z = 0; its end point Q lies in the detector plane, D_od on the far
    # side of the rotation axis; neighbouring columns are du apart along
    # e_u = (-sin, cos, 0) and neighbouring rows dv apart along +z; the
    # middle pixel of an odd detector lies on the line through the source and
    # the origin; rays are ordered [view][row][column]; the generator behind
    # the data agrees.
    V, nu, nv = 5, 9, 7
    du, dv, dso, dod = 0.05, 0.08, 31.25, 15.625
    p0, d = geometry.cone3d_rays(V, nu, nv, du, dv, dso, dod)
    assert p0.shape == (V * nv * nu, 3)
    assert np.allclose(np.linalg.norm(p0[:, :2], axis=1), dso, rtol=1e-14)
    assert np.all(p0[:, 2] == 0.0)
    ph = np.repeat(np.arange(V) * (2 * np.pi / V), nv * nu)
    n = np.stack([np.cos(ph), np.sin(ph), 0 * ph], 1)
    Q = p0 + d
    assert np.allclose(np.einsum("ij,ij->i", Q, n), -dod, atol=1e-12)
    Qg = Q.reshape(V, nv, nu, 3)
    eu = np.stack([-np.sin(ph), np.cos(ph), 0 * ph], 1).reshape(V, nv, nu, 3)
    du_step = np.einsum("vbai,vbai->vba", np.diff(Qg, axis=2), eu[:, :, 1:])
    assert np.allclose(du_step, du, rtol=1e-10)
    assert np.allclose(np.diff(Qg, axis=2)[..., 2], 0.0, atol=1e-14)
    assert np.allclose(np.diff(Qg, axis=1)[..., 2], dv, rtol=1e-10)
    assert np.allclose(np.diff(Qg, axis=1)[..., :2], 0.0, atol=1e-13)
    # central ray: source, origin and middle pixel are collinear
    mid = (np.arange(V) * nv + nv // 2) * nu + nu // 2
    assert np.abs(np.cross(p0[mid], d[mid])).max() <= 1e-12 * dso * (dso + dod)
    assert np.allclose(Q[mid], -dod * n[mid], atol=1e-12)
    # hand-derived pixel: view 1 of 4 (phi = 90 deg), row 0, column nu - 1
    p1, d1 = geometry.cone3d_rays(4, nu, nv, du, dv, dso, dod, views=[1], rows=[0],
                                  cols=[nu - 1])
    ua, vb = (nu - 1) / 2 * du, -(nv - 1) / 2 * dv
    assert np.allclose(p1[0], [0.0, dso, 0.0], atol=1e-13)
    assert np.allclose(p1[0] + d1[0], [-ua, -dod, vb], atol=1e-13)
    sp0, sd = synth.rays_cone3d(V, nu, nv, du, dv, dso, dod)
    assert np.allclose(sp0, p0, atol=1e-13) and np.allclose(sd, d, atol=1e-13)
