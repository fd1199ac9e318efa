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
