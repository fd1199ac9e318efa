"""Grid, FOV mask and point coordinates (Sec. III: E samples f_theta on a
regular grid of coordinates inside a field-of-view mask).

Grid on [-1, 1]^d with N points per axis: pitch h = 2/N, centre of index i
at -1 + (i + 1/2) h.  Arrays are x fastest ([y][x] or [z][y][x]).  The FOV
is the disc x^2 + y^2 <= 1 (2D) or the cylinder x^2 + y^2 <= 1 at every z
(3D).  FOV points are ranked in ascending linear-index order.
"""
import numpy as np


def pitch(N):
    return 2.0 / N


def centres(N):
    return -1.0 + (np.arange(N, dtype=np.float64) + 0.5) * (2.0 / N)


def fov_mask(dim, N):
    c = centres(N)
    disc = (c[None, :] ** 2 + c[:, None] ** 2) <= 1.0
    if dim == 2:
        return disc
    return np.broadcast_to(disc, (N, N, N))


def fov_indices(dim, N):
    """Linear grid indices of the FOV points, ascending (= rank order)."""
    return np.flatnonzero(fov_mask(dim, N).ravel())


def coords(dim, N, idx):
    """Coordinates (x, y[, z]) of the grid points with linear indices idx."""
    idx = np.asarray(idx, dtype=np.int64)
    c = centres(N)
    ix = idx % N
    iy = (idx // N) % N
    if dim == 2:
        return np.stack([c[ix], c[iy]], axis=1)
    iz = idx // (N * N)
    return np.stack([c[ix], c[iy], c[iz]], axis=1)
