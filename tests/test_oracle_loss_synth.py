"""Pins for the FLS ramp filter and for the synthetic-data generator's
closed-form chords (CPU only)."""
import math

import numpy as np

from oracle import loss, step
from paper_2604_09884_amd import synth


def test_ramp_frequency_response_is_ramp():
    # DTFT of the Ram-Lak taps tends to |omega| / (2 pi du) on [-pi, pi]
    du, n = 0.5, 4001
    f = loss.ramp_kernel(n, du)
    j = np.arange(-(n - 1), n)
    for w in np.linspace(-math.pi, math.pi, 21):
        H = np.sum(f * np.cos(w * j))
        assert abs(H - abs(w) / (2 * math.pi * du)) < 2e-4 / du


def test_fls_gradient_fd_and_symmetry():
    rng = np.random.default_rng(0)
    z, y = rng.standard_normal((3, 4, 9)), rng.standard_normal((3, 4, 9))
    du = 0.1
    r = loss.fls_residual(z, y, du)
    g = np.zeros_like(z)
    for idx in np.ndindex(z.shape):
        zp, zm = z.copy(), z.copy()
        zp[idx] += 1e-6
        zm[idx] -= 1e-6
        g[idx] = (loss.fls_loss(zp, y, du) - loss.fls_loss(zm, y, du)) / 2e-6
    assert np.abs(g - r).max() < 1e-6 * np.abs(r).max()
    a, b = rng.standard_normal((2, 2, 9))
    assert abs(np.sum(loss.ramp_filter(a, du) * b) - np.sum(a * loss.ramp_filter(b, du))) < 1e-12


def test_disc_chord_closed_form():
    ph = {"centre": np.array([[0.2, -0.1]]), "axes": np.array([[0.3, 0.3]]),
          "angle": np.array([0.7]), "mu": np.array([2.0])}
    rho = np.linspace(-0.35, 0.35, 71)
    p0 = np.stack([0.2 + rho, np.full_like(rho, -5.0)], 1)
    d = np.tile([0.0, 3.0], (rho.size, 1))
    got = synth.chord_integrals(ph, 2, p0, d)
    ref = 2.0 * 2.0 * np.sqrt(np.maximum(0.09 - rho ** 2, 0))
    # the root gap loses digits only near tangency, where sqrt amplifies rounding
    assert np.abs(got - ref).max() < 1e-6
    inner = np.abs(rho) < 0.29
    assert np.abs(got - ref)[inner].max() < 1e-12


def test_ellipse_area_and_ellipsoid_volume_by_fubini():
    ph = synth.random_ellipses(1, seed=3)
    a, b = ph["axes"][0]
    du = 1e-4
    s = np.arange(-1, 1, du) + du / 2
    p0 = np.stack([s, np.full_like(s, -3.0)], 1)
    d = np.tile([0.0, 1.0], (s.size, 1))
    area = synth.chord_integrals(ph, 2, p0, d).sum() * du / ph["mu"][0]
    assert abs(area - math.pi * a * b) < 1e-5
    ph3 = synth.random_ellipsoids(1, seed=4)
    ax = ph3["axes"][0]
    h = 2e-3
    g = np.arange(-1, 1, h) + h / 2
    X, Z = np.meshgrid(g, g, indexing="ij")
    p0 = np.stack([X.ravel(), np.full(X.size, -3.0), Z.ravel()], 1)
    d = np.tile([0.0, 1.0, 0.0], (X.size, 1))
    vol = synth.chord_integrals(ph3, 3, p0, d).sum() * h * h / ph3["mu"][0]
    assert abs(vol - 4 / 3 * math.pi * np.prod(ax)) < 2e-4


def test_phantoms_inside_fov():
    for seed in range(5):
        e = synth.random_ellipses(10, seed)
        assert np.all(np.linalg.norm(e["centre"], axis=1) + e["axes"].max(1) <= 0.95)
        s = synth.random_ellipsoids(20, seed)
        assert np.all(np.linalg.norm(s["centre"], axis=1) + s["axes"].max(1) <= 0.95)


def test_mse_hand_computed():
    # mean of squared differences over the FOV points only (Sec. IV): FOV =
    # grid indices 0, 2, 3 of a 2 x 2 image; index 1 lies outside and its
    # large difference must not count
    u = np.array([[1.0, 2.0], [3.0, 4.0]])
    ref = np.array([[0.0, 100.0], [5.0, 4.5]])
    fov = np.array([0, 2, 3])
    assert step.mse(u, ref, fov) == (1.0 + 4.0 + 0.25) / 3
    assert step.mse(ref, ref, fov) == 0.0
