"""Scan geometries as explicit ray lists (origin p0, direction d).

The paper's projector P (Sec. III) is a matrix whose rows are discrete ray
integrals; which rays exist is fixed by the scan geometry.  Conventions:

  * 2D parallel beam: view j at angle theta_j = j * span / V; direction
    d = (-sin theta, cos theta); detector axis e = (cos theta, sin theta);
    bin k at s_k = (k - (K-1)/2) du; ray s_k e + t d.  Rays ordered
    [view][bin].
  * 3D circular cone beam: view j at angle phi_j = j * span / V; source
    S = D_so (cos phi, sin phi, 0); detector centre C = -D_od (cos phi,
    sin phi, 0); axes e_u = (-sin phi, cos phi, 0), e_v = (0, 0, 1); pixel
    (a, b) at Q = C + u_a e_u + v_b e_v with u_a = (a - (Nu-1)/2) du and
    v_b = (b - (Nv-1)/2) dv; ray S + t (Q - S).  Rays ordered
    [view][row b][column a].
  * 2D fan beam (the acquisition of Sec. IV-A): the plane z = 0 of the
    cone geometry; view j at angle phi_j = j * span / V; source
    S = D_so (cos phi, sin phi); detector centre C = -D_od (cos phi,
    sin phi); axis e_u = (-sin phi, cos phi); bin a at Q = C + u_a e_u,
    u_a = (a - (K-1)/2) du; ray S + t (Q - S).  Rays ordered [view][bin].
    The paper does not give the source and detector distances; the cone
    world geometry's are used.
"""
import numpy as np


def par2d_rays(n_views, n_bins, du, span=np.pi, views=None):
    views = np.arange(n_views) if views is None else np.atleast_1d(views)
    p0, d = [], []
    for j in views:
        th = j * (span / n_views)
        c, s = np.cos(th), np.sin(th)
        sk = (np.arange(n_bins) - (n_bins - 1) / 2.0) * du
        p0.append(np.stack([sk * c, sk * s], axis=1))
        d.append(np.tile([-s, c], (n_bins, 1)))
    return np.concatenate(p0), np.concatenate(d)


def cone3d_rays(n_views, nu, nv, du, dv, dso, dod, span=2 * np.pi,
                views=None, rows=None, cols=None):
    views = np.arange(n_views) if views is None else np.atleast_1d(views)
    rows = np.arange(nv) if rows is None else np.atleast_1d(rows)
    cols = np.arange(nu) if cols is None else np.atleast_1d(cols)
    p0, d = [], []
    for j in views:
        ph = j * (span / n_views)
        c, s = np.cos(ph), np.sin(ph)
        S = np.array([dso * c, dso * s, 0.0])
        C = np.array([-dod * c, -dod * s, 0.0])
        eu = np.array([-s, c, 0.0])
        ev = np.array([0.0, 0.0, 1.0])
        ua = (cols - (nu - 1) / 2.0) * du
        vb = (rows - (nv - 1) / 2.0) * dv
        Q = C + ua[None, :, None] * eu + vb[:, None, None] * ev
        dd = (Q - S).reshape(-1, 3)
        d.append(dd)
        p0.append(np.tile(S, (dd.shape[0], 1)))
    return np.concatenate(p0), np.concatenate(d)


def fan2d_rays(n_views, n_bins, du, dso, dod, span=2 * np.pi, views=None):
    views = np.arange(n_views) if views is None else np.atleast_1d(views)
    p0, d = [], []
    for j in views:
        ph = j * (span / n_views)
        c, s = np.cos(ph), np.sin(ph)
        S = np.array([dso * c, dso * s])
        C = np.array([-dod * c, -dod * s])
        eu = np.array([-s, c])
        ua = (np.arange(n_bins) - (n_bins - 1) / 2.0) * du
        Q = C[None, :] + ua[:, None] * eu[None, :]
        d.append(Q - S[None, :])
        p0.append(np.tile(S, (n_bins, 1)))
    return np.concatenate(p0), np.concatenate(d)


def problem_rays(problem, views=None):
    """All rays of a configuration (any object with the Problem fields)."""
    if problem.geometry == "par2d":
        return par2d_rays(problem.n_views, problem.n_u, problem.du,
                          problem.view_span, views)
    if problem.geometry == "fan2d":
        return fan2d_rays(problem.n_views, problem.n_u, problem.du,
                          problem.dso, problem.dod, problem.view_span, views)
    return cone3d_rays(problem.n_views, problem.n_u, problem.n_v, problem.du,
                       problem.dv, problem.dso, problem.dod,
                       problem.view_span, views)
