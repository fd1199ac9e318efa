"""Pins for the oracle's multi-resolution hash encoding and the INR built
on it (CPU only): level resolutions, the dense vertex index and the spatial
hash on hand-derived values, partition of unity, exactness at vertices,
reproduction of linear functions on dense levels, continuity across cell
faces, the encoding's adjoint, and the whole INR's Jacobian-transpose
product against central differences."""
import numpy as np
import pytest

from oracle import hashenc, inr
from paper_2604_09884_amd import configs, synth


def _arch(d, levels=3, log2=6, base=2, top=9, W=8, L=2):
    return configs.INRArch("hash", d, 0, 0.0, W, L, hash_levels=levels, hash_feats=2,
                           hash_log2_size=log2, hash_base_res=base, hash_max_res=top)


def _pts(n, d, seed):
    return np.random.default_rng(seed).uniform(-0.999, 0.999, size=(n, d))


def test_resolutions():
    assert hashenc.resolutions(_arch(2, levels=1, base=16, top=16)) == [16]
    assert hashenc.resolutions(_arch(2, levels=16, base=16, top=512))[0] == 16
    assert hashenc.resolutions(_arch(2, levels=16, base=16, top=512))[-1] == 512
    # growth factor 2 from 4 to 32 over 4 levels
    assert hashenc.resolutions(_arch(2, levels=4, base=4, top=32)) == [4, 8, 16, 32]


def test_dense_index_hand_values_and_bijection():
    assert hashenc.vertex_index([[1, 2]], 3, 2, 64)[0] == 9            # 1 + 2*4
    assert hashenc.vertex_index([[2, 0, 3]], 4, 3, 1 << 10)[0] == 77    # 2 + 0*5 + 3*25
    for d, Nl in ((2, 7), (3, 3)):
        g = np.stack(np.meshgrid(*[np.arange(Nl + 1)] * d, indexing="ij"), -1).reshape(-1, d)
        idx = hashenc.vertex_index(g, Nl, d, (Nl + 1) ** d)
        assert np.array_equal(np.sort(idx), np.arange((Nl + 1) ** d))


def test_spatial_hash_hand_values():
    # T = 2^19 < 101^3: hashed.  pi_1 = 0x9E3779B1 -> low 19 bits 0x779B1;
    # pi_2 = 0x30025795 -> low 19 bits 0x25795.
    T, Nl = 1 << 19, 100
    c = np.array([[1, 0, 0], [2, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [3, 0, 0]])
    assert list(hashenc.vertex_index(c, Nl, 3, T)) == [1, 2, 0x779B1, 0x25795, 0x779B0, 3]
    big = np.random.default_rng(3).integers(0, Nl + 1, size=(5000, 3))
    idx = hashenc.vertex_index(big, Nl, 3, T)
    assert idx.min() >= 0 and idx.max() < T


@pytest.mark.parametrize("d", [2, 3])
def test_partition_of_unity_and_vertex_exactness(d):
    a = _arch(d)
    theta = np.ones(inr.n_params(a))
    e = hashenc.encode(theta, _pts(200, d, 1), a)
    assert np.allclose(e, 1.0, atol=1e-14)
    # at a vertex the encoding is that vertex's entry
    theta = np.random.default_rng(2).standard_normal(inr.n_params(a))
    tab = hashenc.tables(theta, a)
    for l, Nl in enumerate(hashenc.resolutions(a)):
        c = np.random.default_rng(4 + l).integers(1, Nl, size=(20, d))
        X = 2.0 * c / Nl - 1.0
        e = hashenc.encode(theta, X, a)[:, 2 * l:2 * l + 2]
        ref = tab[l][hashenc.vertex_index(c, Nl, d, 1 << a.hash_log2_size)]
        assert np.allclose(e, ref, atol=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_dense_levels_reproduce_linear_functions(d):
    # fill every dense level with g(c) = alpha . c + beta (per feature),
    # indexing vertices by the dense formula written out here; multilinear
    # interpolation then returns alpha . p + beta at p = (x + 1) / 2 * N_l
    a = _arch(d, levels=2, log2=12, base=3, top=6)
    T = 1 << 12
    rng = np.random.default_rng(5)
    theta = np.zeros(inr.n_params(a))
    tab = theta[:a.n_table].reshape(2, T, 2)
    coef = rng.standard_normal((2, 2, d + 1))
    for l, Nl in enumerate(hashenc.resolutions(a)):
        assert (Nl + 1) ** d <= T
        g = np.stack(np.meshgrid(*[np.arange(Nl + 1)] * d, indexing="ij"), -1).reshape(-1, d)
        idx = sum(g[:, i] * (Nl + 1) ** i for i in range(d))
        for f in range(2):
            tab[l, idx, f] = g @ coef[l, f, :d] + coef[l, f, d]
    X = _pts(300, d, 6)
    e = hashenc.encode(theta, X, a)
    for l, Nl in enumerate(hashenc.resolutions(a)):
        p = (X + 1.0) / 2.0 * Nl
        for f in range(2):
            assert np.allclose(e[:, 2 * l + f], p @ coef[l, f, :d] + coef[l, f, d], atol=1e-12)


def test_continuous_across_cell_faces():
    a = _arch(3)
    theta = np.random.default_rng(7).standard_normal(inr.n_params(a))
    Nl = hashenc.resolutions(a)[1]
    x0 = 2.0 * 3 / Nl - 1.0                      # a face of level 1's cells
    X = np.array([[x0 - 1e-9, 0.1, -0.2], [x0 + 1e-9, 0.1, -0.2]])
    e = hashenc.encode(theta, X, a)
    assert np.abs(e[0] - e[1]).max() < 1e-6


@pytest.mark.parametrize("d", [2, 3])
def test_encoding_adjoint(d):
    a = _arch(d)
    X = _pts(150, d, 8)
    G = np.random.default_rng(9).standard_normal((150, a.enc_dim))
    t = np.random.default_rng(10).standard_normal(inr.n_params(a))
    lhs = hashenc.encode_vjp(X, G, a) @ t[:a.n_table]
    rhs = np.sum(G * hashenc.encode(t, X, a))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


@pytest.mark.parametrize("d", [2, 3])
def test_inr_vjp_matches_central_differences(d):
    a = _arch(d, W=6, L=2)
    theta, B = synth.random_theta(a, 11)
    X = _pts(40, d, 12)
    cot = np.random.default_rng(13).standard_normal(40)
    g = inr.vjp(theta, B, X, cot, a)
    assert g.size == theta.size == a.n_params
    rng = np.random.default_rng(14)
    sel = np.concatenate([rng.choice(a.n_table, 60, replace=False),
                          a.n_table + np.arange(theta.size - a.n_table)])
    for i in sel:
        e = np.zeros_like(theta)
        e[i] = 1e-6
        fd = (cot @ inr.forward(theta + e, B, X, a) - cot @ inr.forward(theta - e, B, X, a)) / 2e-6
        assert abs(g[i] - fd) <= 1e-6 * (1.0 + abs(fd)), i
