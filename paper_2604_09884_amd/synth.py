"""Seeded synthetic inputs: phantoms, measured data, INR initialisation.

This module generates inputs only.  It holds none of the method's arithmetic
(no grid evaluation, projector, adjoint, gradient or optimiser); both the
HIP path and the FP64 test oracle consume what it produces.

Data follow the paper's recipe for avoiding the inverse crime (Sec. IV-A):
measurements come from a finer model than the reconstruction grid.  Here the
finer model is exact: each ray's value is the closed-form chord length of the
ray through each ellipse/ellipsoid, weighted by its attenuation, so the data
never pass through the discrete projector.

Ray conventions are those stated in ``configs``.
"""
from __future__ import annotations

import math
import os

import numpy as np

from .configs import INRArch, Problem


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------

def random_ellipses(n: int, seed: int, r_max: float = 0.95):
    """n ellipses inside the disc of radius r_max.

    Centre at radius 0.6*sqrt(U) and angle U[0, 2pi); semi-axes U[0.05, 0.35];
    rotation U[0, pi); attenuation U[0.1, 1].  Ellipses that would reach past
    r_max are redrawn.  Returns a dict of arrays.
    """
    rng = np.random.default_rng(seed)
    cen, ax, rot, mu = [], [], [], []
    while len(cen) < n:
        rad = 0.6 * math.sqrt(rng.uniform())
        ang = rng.uniform(0, 2 * math.pi)
        a = rng.uniform(0.05, 0.35, size=2)
        th = rng.uniform(0, math.pi)
        m = rng.uniform(0.1, 1.0)
        if rad + a.max() > r_max:
            continue
        cen.append([rad * math.cos(ang), rad * math.sin(ang)])
        ax.append(a)
        rot.append(th)
        mu.append(m)
    return {"centre": np.array(cen), "axes": np.array(ax),
            "angle": np.array(rot), "mu": np.array(mu)}


def _quat_to_rot(q):
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def random_ellipsoids(n: int, seed: int, r_max: float = 0.95):
    """n ellipsoids inside the ball of radius r_max (hence inside the FOV
    cylinder and the grid).  Centre uniform in the ball of radius 0.6;
    semi-axes U[0.05, 0.35]; rotation from a normalised Gaussian quaternion;
    attenuation U[0.1, 1]."""
    rng = np.random.default_rng(seed)
    cen, ax, rots, mu = [], [], [], []
    while len(cen) < n:
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        rad = 0.6 * rng.uniform() ** (1.0 / 3.0)
        a = rng.uniform(0.05, 0.35, size=3)
        R = _quat_to_rot(rng.normal(size=4))
        m = rng.uniform(0.1, 1.0)
        if rad + a.max() > r_max:
            continue
        cen.append(rad * v)
        ax.append(a)
        rots.append(R)
        mu.append(m)
    return {"centre": np.array(cen), "axes": np.array(ax),
            "rot": np.array(rots), "mu": np.array(mu)}


def ellipse_rot2(angle):
    c, s = math.cos(angle), math.sin(angle)
    return np.array([[c, -s], [s, c]])


def phantom(problem: Problem):
    if problem.dim == 2:
        return random_ellipses(problem.n_ellipses, problem.seed_phantom)
    return random_ellipsoids(problem.n_ellipses, problem.seed_phantom)


def _rotations(ph, dim):
    if dim == 2:
        return np.stack([ellipse_rot2(a) for a in ph["angle"]])
    return ph["rot"]


def chord_integrals(ph, dim: int, p0: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Sum over shapes of mu * (length of the ray p0 + t d inside the shape).

    The ray is mapped into each shape's unit-ball frame q(t) = A^-1 R^T
    (p0 + t d - c); |q(t)|^2 = 1 is a quadratic a t^2 + b t + c0 = 0 whose
    root gap sqrt(b^2 - 4 a c0)/a, times |d|, is the chord length."""
    p0 = np.asarray(p0, np.float64)
    d = np.asarray(d, np.float64)
    out = np.zeros(p0.shape[0])
    dn = np.linalg.norm(d, axis=1)
    dh = d / dn[:, None]
    rots = _rotations(ph, dim)
    for cen, ax, R, mu in zip(ph["centre"], ph["axes"], rots, ph["mu"]):
        # only rays passing within the largest semi-axis of the centre can
        # meet the shape (it lies inside that ball)
        w = cen - p0
        wd = np.einsum("ij,ij->i", w, dh)
        near = np.einsum("ij,ij->i", w, w) - wd * wd <= (1.0 + 1e-9) * float(np.max(ax)) ** 2
        sel = np.nonzero(near)[0]
        if sel.size == 0:
            continue
        q0 = ((p0[sel] - cen) @ R) / ax
        qd = (d[sel] @ R) / ax
        a = np.einsum("ij,ij->i", qd, qd)
        b = 2 * np.einsum("ij,ij->i", q0, qd)
        c0 = np.einsum("ij,ij->i", q0, q0) - 1
        disc = b * b - 4 * a * c0
        ok = disc > 0
        chord = np.zeros_like(a)
        chord[ok] = np.sqrt(disc[ok]) / a[ok] * dn[sel][ok]
        out[sel] += mu * chord
    return out


def raster(ph, dim: int, N: int) -> np.ndarray:
    """Point-sampled phantom at grid centres (the MSE ground truth).  Every
    shape lies inside radius 0.95, so the raster vanishes outside the FOV.
    Shape [N]*dim, x fastest."""
    c = -1 + (np.arange(N) + 0.5) * (2.0 / N)
    rots = _rotations(ph, dim)
    if dim == 2:
        Y, X = np.meshgrid(c, c, indexing="ij")
        P = np.stack([X, Y], -1).reshape(-1, 2)
    else:
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        P = np.stack([X, Y, Z], -1).reshape(-1, 3)
    img = np.zeros(P.shape[0])
    for cen, ax, R, mu in zip(ph["centre"], ph["axes"], rots, ph["mu"]):
        q = ((P - cen) @ R) / ax
        img += mu * (np.einsum("ij,ij->i", q, q) <= 1.0)
    return img.reshape([N] * dim)


# --------------------------------------------------------------------------
# ray sets (for the analytic data only)
# --------------------------------------------------------------------------

def rays_par2d(n_views, n_bins, du, span=math.pi, views=None):
    """Parallel-beam rays, view-major then bin: (p0, d) with |d| = 1."""
    views = np.arange(n_views) if views is None else np.asarray(views)
    th = views * (span / n_views)
    s = (np.arange(n_bins) - (n_bins - 1) / 2.0) * du
    c, sn = np.cos(th)[:, None], np.sin(th)[:, None]
    p0 = np.stack([s[None, :] * c, s[None, :] * sn], -1)
    d = np.stack([-sn + 0 * s[None, :], c + 0 * s[None, :]], -1)
    return p0.reshape(-1, 2), d.reshape(-1, 2)


def rays_cone3d(n_views, nu, nv, du, dv, dso, dod, span=2 * math.pi,
                views=None, rows=None):
    """Cone-beam rays ordered [view][row b][column a]: (S, Q - S)."""
    views = np.arange(n_views) if views is None else np.asarray(views)
    rows = np.arange(nv) if rows is None else np.asarray(rows)
    ph = views * (span / n_views)
    u = (np.arange(nu) - (nu - 1) / 2.0) * du
    v = (rows - (nv - 1) / 2.0) * dv
    out_p, out_d = [], []
    for p in ph:
        c, s = math.cos(p), math.sin(p)
        S = np.array([dso * c, dso * s, 0.0])
        C = np.array([-dod * c, -dod * s, 0.0])
        eu = np.array([-s, c, 0.0])
        ev = np.array([0.0, 0.0, 1.0])
        Q = C[None, None, :] + u[None, :, None] * eu + v[:, None, None] * ev
        dd = (Q - S).reshape(-1, 3)
        out_d.append(dd)
        out_p.append(np.broadcast_to(S, dd.shape))
    return np.concatenate(out_p), np.concatenate(out_d)


def rays_fan2d(n_views, n_bins, du, dso, dod, span=2 * math.pi, views=None):
    """Fan-beam rays ordered [view][bin]: (S, Q - S), the z = 0 plane of the
    cone geometry."""
    views = np.arange(n_views) if views is None else np.asarray(views)
    ph = views * (span / n_views)
    u = (np.arange(n_bins) - (n_bins - 1) / 2.0) * du
    c, s = np.cos(ph)[:, None], np.sin(ph)[:, None]
    Sx, Sy = dso * c + 0 * u[None, :], dso * s + 0 * u[None, :]
    Qx, Qy = -dod * c - u[None, :] * s, -dod * s + u[None, :] * c
    p0 = np.stack([Sx, Sy], -1).reshape(-1, 2)
    d = np.stack([Qx - Sx, Qy - Sy], -1).reshape(-1, 2)
    return p0, d


def rays(problem: Problem, views=None):
    if problem.geometry == "par2d":
        return rays_par2d(problem.n_views, problem.n_u, problem.du,
                          problem.view_span, views)
    if problem.geometry == "fan2d":
        return rays_fan2d(problem.n_views, problem.n_u, problem.du, problem.dso,
                          problem.dod, problem.view_span, views)
    return rays_cone3d(problem.n_views, problem.n_u, problem.n_v, problem.du,
                       problem.dv, problem.dso, problem.dod,
                       problem.view_span, views)


def sinogram(problem: Problem, ph=None, noisy: bool = True) -> np.ndarray:
    """Measured data y, FP64, shape [V][K] (2D) or [V][Nv][Nu] (3D)."""
    ph = phantom(problem) if ph is None else ph

    def one(j):
        p0, d = rays(problem, views=[j])
        return chord_integrals(ph, problem.dim, p0, d)
    if problem.n_rays > 200000:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(min(16, os.cpu_count() or 4)) as ex:
            out = list(ex.map(one, range(problem.n_views)))
    else:
        out = [one(j) for j in range(problem.n_views)]
    y = np.concatenate(out)
    if noisy and problem.photons > 0:
        rng = np.random.default_rng(problem.seed_noise)
        counts = rng.poisson(problem.photons * np.exp(-y))
        y = -np.log(np.maximum(counts, 1) / problem.photons)
    shape = ((problem.n_views, problem.n_u) if problem.dim == 2 else
             (problem.n_views, problem.n_v, problem.n_u))
    return y.reshape(shape)


# --------------------------------------------------------------------------
# INR initialisation
# --------------------------------------------------------------------------

def init_inr(arch: INRArch, seed: int):
    """Initial parameters theta (FP64 flat) and Fourier matrix B ([F][d]).

    Flat layout: for each affine layer in order, W (fan_out x fan_in,
    row-major) then b; the output layer last.  FFN: Xavier-uniform weights,
    zero biases, B ~ N(0, sigma^2).  SIREN: first layer U(+-1/fan_in), the
    others U(+-sqrt(6/fan_in)/omega0), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    if arch.kind == "hash":  # tables U(+-1e-4), as in the hash-encoding paper
        parts.append(rng.uniform(-1e-4, 1e-4, size=arch.n_table))
    for li, (fi, fo) in enumerate(arch.layer_dims()):
        if arch.kind != "siren":
            lim = math.sqrt(6.0 / (fi + fo))
        else:
            lim = 1.0 / fi if li == 0 else math.sqrt(6.0 / fi) / arch.omega0
        parts.append(rng.uniform(-lim, lim, size=fi * fo))
        parts.append(np.zeros(fo))
    theta = np.concatenate(parts)
    if arch.kind == "ffn":
        B = rng.normal(0.0, arch.sigma, size=(arch.n_freq, arch.in_dim))
    else:
        B = np.zeros((0, arch.in_dim))
    return theta, B


def random_theta(arch: INRArch, seed: int, bias_scale: float = 0.1):
    """Initial parameters with non-zero biases (for tests that must exercise
    every bias gradient)."""
    theta, B = init_inr(arch, seed)
    rng = np.random.default_rng(seed + 7)
    if arch.kind == "hash":  # tables large enough to matter
        theta[:arch.n_table] = rng.uniform(-0.5, 0.5, size=arch.n_table)
    off = arch.n_table
    for fi, fo in arch.layer_dims():
        off += fi * fo
        theta[off:off + fo] = rng.uniform(-bias_scale, bias_scale, size=fo)
        off += fo
    return theta, B


def uniform_subset(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct ranks in [0, n), ascending (test input only)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=k, replace=False))
