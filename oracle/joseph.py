"""Joseph's ray-driven projector P and its exact transpose (Sec. III: P is a
discrete forward-projection matrix in R^{m x n}; v = P^T r).

Method (Joseph, "An improved algorithm for reprojecting rays through pixel
images", IEEE TMI 1982): each ray is sampled once per grid slice along its
principal axis; at each slice the image is linearly (2D) or bilinearly (3D)
interpolated at the crossing point; the sum is multiplied by the step length
between slices, h |d| / |d_axis|.

Readings of points the paper leaves open (the paper uses a third-party
library for P):
  * principal axis: y if |d_y| >= (1 - tau) |d_x| with tau = 1e-9, else x,
    decided in float64 (3D rays must have |d_z| below the in-plane
    component; all cone geometries here satisfy it);
  * every one of the N slices is visited; interpolation outside the grid
    reads zero (zero padding);
  * fractional index of a coordinate q along an axis: phi = (q + 1)/h - 1/2,
    taps floor(phi) with weight 1 - w and floor(phi) + 1 with weight w,
    w = phi - floor(phi).

The matrix is assembled as (ray, voxel, weight) triplets; P u and P^T r are
then plain sparse products, so P^T is the transpose of P exactly.
"""
import numpy as np
import scipy.sparse as sp

from .grid import centres

TAU = 1e-9


def y_principal(d):
    d = np.asarray(d, np.float64)
    return np.abs(d[:, 1]) >= (1.0 - TAU) * np.abs(d[:, 0])


def _linear_taps(phi):
    i0 = np.floor(phi)
    w = phi - i0
    i0 = i0.astype(np.int64)
    return ((i0, 1.0 - w), (i0 + 1, w))


def triplets(N, dim, p0, d):
    """Nonzeros of the projector rows for the given rays.

    Returns (ray, voxel, weight) arrays; voxel is the linear index into the
    grid ([y][x] or [z][y][x]).  Taps outside the grid are dropped (they
    would multiply a zero-padded value)."""
    p0 = np.asarray(p0, np.float64)
    d = np.asarray(d, np.float64)
    h = 2.0 / N
    c = centres(N)
    ypr = y_principal(d)
    if dim == 3 and not np.all(np.abs(d[:, 2]) < np.maximum(np.abs(d[:, 0]),
                                                           np.abs(d[:, 1]))):
        raise ValueError("ray too steep in z for an in-plane principal axis")
    out_r, out_v, out_w = [], [], []
    for axis in (1, 0):
        sel = np.flatnonzero(ypr if axis == 1 else ~ypr)
        if sel.size == 0:
            continue
        other = 1 - axis
        P0, D = p0[sel], d[sel]
        # crossing of each ray with every slice plane {q_axis = c(i)}
        t = (c[None, :] - P0[:, axis:axis + 1]) / D[:, axis:axis + 1]
        step = h * np.linalg.norm(D, axis=1) / np.abs(D[:, axis])
        slice_idx = np.broadcast_to(np.arange(N), t.shape)
        ray_idx = np.broadcast_to(sel[:, None], t.shape)
        q_other = P0[:, other:other + 1] + t * D[:, other:other + 1]
        taps_o = _linear_taps((q_other + 1.0) / h - 0.5)
        if dim == 2:
            for io, wo in taps_o:
                ok = (io >= 0) & (io < N)
                if axis == 1:
                    vox = slice_idx * N + io      # row y = slice, column x = io
                else:
                    vox = io * N + slice_idx      # row y = io, column x = slice
                out_r.append(ray_idx[ok])
                out_v.append(vox[ok])
                out_w.append((wo * step[:, None])[ok])
        else:
            q_z = P0[:, 2:3] + t * D[:, 2:3]
            taps_z = _linear_taps((q_z + 1.0) / h - 0.5)
            for io, wo in taps_o:
                for iz, wz in taps_z:
                    ok = (io >= 0) & (io < N) & (iz >= 0) & (iz < N)
                    if axis == 1:
                        vox = (iz * N + slice_idx) * N + io
                    else:
                        vox = (iz * N + io) * N + slice_idx
                    out_r.append(ray_idx[ok])
                    out_v.append(vox[ok])
                    out_w.append((wo * wz * step[:, None])[ok])
    return (np.concatenate(out_r), np.concatenate(out_v),
            np.concatenate(out_w))


def system_matrix(N, dim, p0, d):
    """P for the given rays as a CSR matrix of shape (rays, N^dim)."""
    r, v, w = triplets(N, dim, p0, d)
    m = np.asarray(p0).shape[0]
    return sp.csr_matrix((w, (r, v)), shape=(m, N ** dim))


def problem_matrix(problem):
    """P for every ray of a configuration, assembled view by view."""
    from .geometry import problem_rays
    blocks = []
    for j in range(problem.n_views):
        p0, d = problem_rays(problem, views=[j])
        blocks.append(system_matrix(problem.N, problem.dim, p0, d))
    return sp.vstack(blocks, format="csr")


def project(u, N, dim, p0, d):
    return system_matrix(N, dim, p0, d) @ np.asarray(u, np.float64).ravel()


def backproject(r, N, dim, p0, d):
    A = system_matrix(N, dim, p0, d)
    return (A.T @ np.asarray(r, np.float64).ravel()).reshape([N] * dim)


def voxel_weights(N, dim, p0, d, vox):
    """P[ray, vox] for each ray, computed from the single slice of the ray
    that can touch the voxel (the voxel's index along the ray's principal
    axis).  Same definition as ``triplets``, restricted to one slice; used to
    evaluate entries of P^T r at a few voxels of grids too large for the full
    matrix."""
    p0 = np.asarray(p0, np.float64)
    d = np.asarray(d, np.float64)
    h = 2.0 / N
    c = centres(N)
    ix = vox % N
    iy = (vox // N) % N
    iz = vox // (N * N)
    ypr = y_principal(d)
    out = np.zeros(p0.shape[0])
    for axis in (1, 0):
        sel = np.flatnonzero(ypr if axis == 1 else ~ypr)
        if sel.size == 0:
            continue
        other = 1 - axis
        P0, D = p0[sel], d[sel]
        s_idx, o_idx = (iy, ix) if axis == 1 else (ix, iy)
        t = (c[s_idx] - P0[:, axis]) / D[:, axis]
        step = h * np.linalg.norm(D, axis=1) / np.abs(D[:, axis])
        phi_o = (P0[:, other] + t * D[:, other] + 1.0) / h - 0.5
        wt = np.zeros(sel.size)
        for io, wo in _linear_taps(phi_o):
            wt += np.where(io == o_idx, wo, 0.0)
        if dim == 3:
            phi_z = (P0[:, 2] + t * D[:, 2] + 1.0) / h - 0.5
            wz = np.zeros(sel.size)
            for iz0, w0 in _linear_taps(phi_z):
                wz += np.where(iz0 == iz, w0, 0.0)
            wt = wt * wz
        out[sel] = wt * step
    return out
