"""Pins for the oracle's ordered subsets over views (CPU only): the subsets
partition the views, a subset's rows are exactly the projector built from
that subset's rays alone, the subset losses and gradients add up to the
full ones (LS and FLS), one subset is the plain step, and the subset
gradient is the finite-difference gradient of the subset loss."""
import numpy as np
import pytest

from oracle import geometry, joseph, step
from paper_2604_09884_amd import configs, synth

ARCH = configs.INRArch("ffn", 2, 3, 2.0, 6, 2)


def _cases():
    return [configs.par2d_problem(10, 12, 15, arch=ARCH),
            configs.fan2d_problem(10, 9, 15, arch=ARCH),
            configs.cone_problem(6, 5, 8, arch=configs.INRArch("ffn", 3, 3, 1.5, 6, 2))]


def test_subsets_partition_the_views():
    for V, S in ((20, 4), (20, 3), (7, 7), (9, 1)):
        allv = np.concatenate([step.subset_views(V, S, s) for s in range(S)])
        assert np.array_equal(np.sort(allv), np.arange(V))
        for s in range(S):
            assert np.all(step.subset_views(V, S, s) % S == s)


@pytest.mark.parametrize("cfg", _cases(), ids=["par2d", "fan2d", "cone3d"])
def test_subset_rows_equal_projector_of_subset_rays(cfg):
    prob = step.Problem(cfg)
    for S in (2, 3):
        for s in range(S):
            views = step.subset_views(cfg.n_views, S, s)
            sub, rows = step.subset_problem(prob, views)
            p0, d = geometry.problem_rays(cfg, views=views)
            A = joseph.system_matrix(cfg.N, cfg.dim, p0, d)
            assert (abs(sub.P - A)).max() == 0


@pytest.mark.parametrize("kind", ["ls", "fls"])
@pytest.mark.parametrize("cfg", _cases(), ids=["par2d", "fan2d", "cone3d"])
def test_subset_losses_and_gradients_add_up(cfg, kind):
    prob = step.Problem(cfg)
    th, B = synth.random_theta(cfg.arch, 41)
    y = np.random.default_rng(42).standard_normal(prob.P.shape[0])
    g_full, L_full, *_ = step.grad_estimate(prob, th, B, y, prob.fov, kind)
    S = 3
    g_sum, L_sum = np.zeros_like(g_full), 0.0
    for s in range(S):
        sub, rows = step.subset_problem(prob, step.subset_views(cfg.n_views, S, s))
        g, L, *_ = step.grad_estimate(sub, th, B, y[rows], prob.fov, kind)
        g_sum += g
        L_sum += L
    assert abs(L_sum - L_full) <= 1e-12 * abs(L_full)
    assert np.linalg.norm(g_sum - g_full) <= 1e-12 * np.linalg.norm(g_full)
    # one subset is the plain problem
    sub, rows = step.subset_problem(prob, step.subset_views(cfg.n_views, 1, 0))
    assert np.array_equal(rows, np.arange(prob.P.shape[0]))
    g1, L1, *_ = step.grad_estimate(sub, th, B, y, prob.fov, kind)
    assert L1 == L_full and np.array_equal(g1, g_full)


def test_subset_gradient_is_gradient_of_subset_loss():
    cfg = configs.par2d_problem(8, 6, 11, arch=ARCH)
    prob = step.Problem(cfg)
    th, B = synth.random_theta(ARCH, 43)
    y = np.random.default_rng(44).standard_normal(prob.P.shape[0])
    views = step.subset_views(cfg.n_views, 3, 1)
    sub, rows = step.subset_problem(prob, views)
    p0, d = geometry.problem_rays(cfg, views=views)
    A = joseph.system_matrix(cfg.N, 2, p0, d)

    def L(t):
        return 0.5 * np.sum((A @ prob.E(t, B) - y[rows]) ** 2)
    g, *_ = step.grad_estimate(sub, th, B, y[rows], prob.fov)
    fd = np.array([(L(th + e) - L(th - e)) / 2e-6 for e in 1e-6 * np.eye(th.size)])
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)
