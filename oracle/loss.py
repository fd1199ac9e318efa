"""Data-fidelity losses and their z-gradients (Sec. II; Sec. III, note after
Algorithm 1).

  LS:  L(z, y) = 1/2 ||z - y||^2,              dL/dz = z - y
  FLS: L(z, y) = 1/2 (z - y)^T F (z - y),       dL/dz = F (z - y)

F is a convolution with a ramp filter along the detector direction of each
projection row (the filter of filtered backprojection).  Reading for the
kernel: the band-limited ramp of Ramachandran and Lakshminarayanan (Kak and
Slaney, Principles of Computerized Tomographic Imaging, Eq. 3.61) in units of
the detector pitch du:
  f[0] = 1/(4 du),  f[j] = -1/(pi^2 j^2 du) for odd j,  0 for even j != 0,
applied as the linear (zero-padded, not circular) convolution over the
detector-u index of every (view, row).  It is symmetric, so F^T = F and the
gradient above holds.
"""
import numpy as np


def ls_residual(z, y):
    return np.asarray(z, np.float64) - np.asarray(y, np.float64)


def ls_loss(z, y):
    r = ls_residual(z, y)
    return 0.5 * float(np.dot(r.ravel(), r.ravel()))


def ramp_kernel(n_u, du):
    """Ram-Lak taps f[j] for j = -(n_u-1) .. n_u-1."""
    j = np.arange(-(n_u - 1), n_u)
    f = np.zeros(j.size)
    f[j == 0] = 1.0 / (4.0 * du)
    odd = (j % 2) != 0
    f[odd] = -1.0 / (np.pi ** 2 * j[odd].astype(np.float64) ** 2 * du)
    return f


def ramp_filter(q, du):
    """F q: linear convolution with the ramp along the last axis."""
    q = np.asarray(q, np.float64)
    n_u = q.shape[-1]
    f = ramp_kernel(n_u, du)
    flat = q.reshape(-1, n_u)
    out = np.empty_like(flat)
    for i in range(flat.shape[0]):
        out[i] = np.convolve(flat[i], f, mode="full")[n_u - 1:2 * n_u - 1]
    return out.reshape(q.shape)


def fls_residual(z, y, du):
    return ramp_filter(ls_residual(z, y), du)


def fls_loss(z, y, du):
    q = ls_residual(z, y)
    return 0.5 * float(np.dot(q.ravel(), ramp_filter(q, du).ravel()))
