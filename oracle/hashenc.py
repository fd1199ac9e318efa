"""Multi-resolution hash encoding (the third INR of Sec. IV, after Mueller
et al., "Instant neural graphics primitives with a multiresolution hash
encoding", 2022), as the first stage of an INR whose MLP is the FFN's
ReLU network.

Readings (the paper names the architecture and gives none of its sizes):
  * a point x in [-1, 1]^d is mapped to y = (x + 1) / 2 in [0, 1]^d;
  * level l = 0..Lh-1 has resolution N_l = floor(N_min * b^l + 1e-6)
    with b = exp((ln N_max - ln N_min) / (Lh - 1)) (b = 1 for one level;
    the 1e-6 keeps N_{Lh-1} = N_max under rounding); its grid vertices are
    c in {0..N_l}^d;
  * at level l the point lies at p = y * N_l; the 2^d vertices of its cell
    are floor(p) + delta, delta in {0, 1}^d (a point on the upper face of
    the domain uses the cell below), with multilinear weights
    prod_i (delta_i ? f_i : 1 - f_i), f = p - floor(p);
  * vertex index in the level's table of T entries: if (N_l + 1)^d <= T,
    the dense index sum_i c_i (N_l + 1)^i; otherwise the spatial hash
    (XOR_i c_i * pi_i) mod T in 32-bit unsigned arithmetic, pi = (1,
    2654435761, 805459861);
  * each entry holds F features; the encoding is the concatenation over
    levels of the interpolated features (level-major, K = Lh * F values).

Parameter layout: the tables first ([Lh][T][F], level-major), then the MLP
in the usual layout.
"""
import math

import numpy as np

PRIMES = (1, 2654435761, 805459861)


def resolutions(arch):
    L = arch.hash_levels
    n0, n1 = arch.hash_base_res, arch.hash_max_res
    b = 1.0 if L == 1 else math.exp((math.log(n1) - math.log(n0)) / (L - 1))
    return [int(math.floor(n0 * b ** l + 1e-6)) for l in range(L)]


def table_size(arch):
    return 1 << arch.hash_log2_size


def n_table_params(arch):
    return arch.hash_levels * table_size(arch) * arch.hash_feats


def vertex_index(c, Nl, d, T):
    """Table index of integer vertices c (n x d) at a level of resolution Nl."""
    c = np.asarray(c, np.int64)
    if (Nl + 1) ** d <= T:
        idx = np.zeros(c.shape[0], np.int64)
        for i in range(d - 1, -1, -1):
            idx = idx * (Nl + 1) + c[:, i]
        return idx
    h = np.zeros(c.shape[0], np.uint64)
    for i in range(d):
        h ^= (c[:, i].astype(np.uint64) * np.uint64(PRIMES[i])) & np.uint64(0xFFFFFFFF)
    return (h % np.uint64(T)).astype(np.int64)


def corners(X, Nl):
    """Vertices (n x 2^d x d) and weights (n x 2^d) of the points' cells."""
    X = np.asarray(X, np.float64)
    n, d = X.shape
    p = (X + 1.0) / 2.0 * Nl
    base = np.minimum(np.floor(p), Nl - 1).astype(np.int64)
    f = p - base
    verts = np.zeros((n, 1 << d, d), np.int64)
    w = np.ones((n, 1 << d))
    for m in range(1 << d):
        for i in range(d):
            bit = (m >> i) & 1
            verts[:, m, i] = base[:, i] + bit
            w[:, m] *= f[:, i] if bit else 1.0 - f[:, i]
    return verts, w


def tables(theta, arch):
    T, F = table_size(arch), arch.hash_feats
    n = n_table_params(arch)
    return np.asarray(theta[:n], np.float64).reshape(arch.hash_levels, T, F)


def encode(theta, X, arch):
    """The K = Lh * F encoding values of each point (n x K)."""
    X = np.asarray(X, np.float64)
    d, T, F = X.shape[1], table_size(arch), arch.hash_feats
    tab = tables(theta, arch)
    out = []
    for l, Nl in enumerate(resolutions(arch)):
        verts, w = corners(X, Nl)
        enc = np.zeros((X.shape[0], F))
        for m in range(1 << d):
            idx = vertex_index(verts[:, m, :], Nl, d, T)
            enc += w[:, m:m + 1] * tab[l][idx]
        out.append(enc)
    return np.concatenate(out, axis=1)


def encode_vjp(X, g_enc, arch):
    """Gradient of sum_i g_enc[i] . encode(x_i) with respect to the tables,
    flat in the parameter layout (the encoding is linear in the tables)."""
    X = np.asarray(X, np.float64)
    d, T, F = X.shape[1], table_size(arch), arch.hash_feats
    g = np.zeros((arch.hash_levels, T, F))
    for l, Nl in enumerate(resolutions(arch)):
        verts, w = corners(X, Nl)
        ge = g_enc[:, l * F:(l + 1) * F]
        for m in range(1 << d):
            idx = vertex_index(verts[:, m, :], Nl, d, T)
            np.add.at(g[l], idx, w[:, m:m + 1] * ge)
    return g.ravel()
