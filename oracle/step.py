"""Algorithm 1 (stochastic gradient estimation) followed by an Adam update.

Steps, in the paper's order:
  1. z = P E{f_theta}                      (no gradient tracking)
  2. v = P^T dL/dz(z, y)                   (LS: z - y; FLS: F (z - y))
  3. draw I subset of [n]                  (passed in, or from ``sampler``)
  4. virtual loss L~ = (n/|I|) sum_{i in I} v_i f_theta(x_i)       (Eq. (3))
  5. grad L~ = (n/|I|) sum_{i in I} v_i grad f_theta(x_i)          (Eq. (2))
then theta <- Adam(theta, grad L~).
With ordered subsets, P, y and the loss of steps 1-2 are those of the
step's view subset (``subset_problem``).

Here P is an explicit sparse matrix (``joseph.problem_matrix``) and step 5 is
the exact reverse-mode sum of ``inr.vjp`` with cotangent (n/|I|) v_I.
"""
import numpy as np

from . import adam, grid, inr, loss


class Problem:
    """Everything Algorithm 1 needs about one reconstruction problem."""

    def __init__(self, cfg, P=None):
        self.cfg = cfg
        self.arch = cfg.arch
        self.dim, self.N = cfg.dim, cfg.N
        self.fov = grid.fov_indices(cfg.dim, cfg.N)
        self.n = self.fov.size
        self.X = grid.coords(cfg.dim, cfg.N, self.fov)
        if P is None:
            from .joseph import problem_matrix
            P = problem_matrix(cfg)
        self.P = P

    def E(self, theta, B):
        u = np.zeros(self.N ** self.dim)
        u[self.fov] = inr.forward(theta, B, self.X, self.arch)
        return u

    def residual(self, z, y, kind="ls"):
        y = np.asarray(y, np.float64).ravel()
        if kind == "ls":
            r = loss.ls_residual(z, y)
            return r, 0.5 * float(r @ r)
        shape = (-1, self.cfg.n_u)
        q = loss.ls_residual(z, y)
        r = loss.ramp_filter(q.reshape(shape), self.cfg.du).ravel()
        return r, 0.5 * float(q @ r)


def full_gradient(prob, theta, B, y, kind="ls"):
    """Exact grad L(theta) = sum_{i=1}^n v_i grad f(x_i) (Sec. III)."""
    u = prob.E(theta, B)
    z = prob.P @ u
    r, L = prob.residual(z, y, kind)
    v = prob.P.T @ r
    return inr.vjp(theta, B, prob.X, v[prob.fov], prob.arch), L


def grad_estimate(prob, theta, B, y, idx, kind="ls", v=None):
    """Eq. (2) for the index set idx (grid linear indices inside the FOV).
    Returns (g, L, u, z, r, v)."""
    u = prob.E(theta, B)
    z = prob.P @ u
    r, L = prob.residual(z, y, kind)
    if v is None:
        v = prob.P.T @ r
    idx = np.asarray(idx, np.int64)
    scale = prob.n / idx.size
    X = grid.coords(prob.dim, prob.N, idx)
    g = inr.vjp(theta, B, X, scale * v[idx], prob.arch)
    return g, L, u, z, r, v


def grad_step(prob, theta, B, m, vstate, t, y, idx, lr, kind="ls",
              beta1=0.9, beta2=0.999, eps=1e-8):
    """One Algorithm-1 gradient estimate and one Adam step (t is 1-based).
    Returns (theta', m', v', loss, ||g||^2)."""
    g, L, *_ = grad_estimate(prob, theta, B, y, idx, kind)
    theta2, m2, v2 = adam.adam_update(theta, m, vstate, g, t, lr, beta1,
                                      beta2, eps)
    return theta2, m2, v2, L, float(g @ g)


def subset_views(n_views, n_subsets, s):
    """Ordered subsets over views (end of Sec. III: the gradient may be taken
    with respect to a subset of the views).  Reading: S interleaved subsets,
    subset s holding views j with j mod S == s, and step t using subset
    t mod S."""
    return np.arange(s, n_views, n_subsets)


def subset_problem(prob, views):
    """The problem restricted to the listed views: the rows of P that belong
    to them (rays are view-major, so each view's rows are contiguous), in
    view order.  Returns (Problem, rows); the data of the subset is
    y[rows]."""
    views = np.asarray(views, np.int64)
    per_view = prob.P.shape[0] // prob.cfg.n_views
    rows = (views[:, None] * per_view + np.arange(per_view)[None, :]).ravel()
    return Problem(prob.cfg, P=prob.P[rows]), rows


def mse(u, u_true, fov):
    """Pixel-wise MSE over the FOV points (Sec. IV-A, IV-B)."""
    d = np.asarray(u, np.float64).ravel()[fov] - np.asarray(u_true).ravel()[fov]
    return float(d @ d) / fov.size
