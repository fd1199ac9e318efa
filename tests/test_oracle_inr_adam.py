"""Pins for the oracle INR, its Jacobian-transpose product, Eq. (2)'s
estimator and Adam (CPU only)."""
import itertools
import math

import numpy as np
import pytest
import torch

from oracle import adam, grid, inr, joseph, step
from paper_2604_09884_amd import configs, synth

FFN = configs.INRArch("ffn", 2, 3, 2.0, 6, 2)
SIREN = configs.INRArch("siren", 2, 0, 0.0, 5, 3, omega0=3.0)
FFN3 = configs.INRArch("ffn", 3, 4, 1.5, 8, 3)


def _theta(arch, seed):
    th, B = synth.random_theta(arch, seed)
    return th, B


def test_forward_hand_computed():
    # FFN with one frequency, width 2, one hidden layer, written out by hand
    arch = configs.INRArch("ffn", 2, 1, 1.0, 2, 1)
    B = np.array([[0.25, -0.5]])
    W1 = np.array([[1.0, -2.0], [0.5, 3.0]])
    b1 = np.array([0.1, -0.2])
    w2 = np.array([[2.0, -1.0]])
    b2 = np.array([0.3])
    theta = np.concatenate([W1.ravel(), b1, w2.ravel(), b2])
    x = np.array([[0.2, 0.4]])
    phase = 2 * math.pi * (0.25 * 0.2 - 0.5 * 0.4)
    a0 = np.array([math.sin(phase), math.cos(phase)])
    h = np.maximum(W1 @ a0 + b1, 0)
    ref = 2.0 * h[0] - 1.0 * h[1] + 0.3
    assert abs(inr.forward(theta, B, x, arch)[0] - ref) < 1e-15


def test_siren_forward_hand_computed():
    # SIREN with width 2, two sine layers and omega0 = 2.5, written out by
    # hand: a_l = sin(omega0 (W_l a_{l-1} + b_l)), f = w . a_2 + b
    arch = configs.INRArch("siren", 2, 0, 0.0, 2, 2, omega0=2.5)
    W1 = np.array([[0.7, -0.3], [0.2, 0.9]])
    b1 = np.array([0.05, -0.1])
    W2 = np.array([[-0.4, 0.6], [1.1, 0.25]])
    b2 = np.array([0.2, 0.0])
    w3 = np.array([[1.5, -0.8]])
    b3 = np.array([-0.25])
    theta = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3.ravel(), b3])
    x0, x1 = -0.3, 0.6
    h0 = math.sin(2.5 * (0.7 * x0 - 0.3 * x1 + 0.05))
    h1 = math.sin(2.5 * (0.2 * x0 + 0.9 * x1 - 0.1))
    g0 = math.sin(2.5 * (-0.4 * h0 + 0.6 * h1 + 0.2))
    g1 = math.sin(2.5 * (1.1 * h0 + 0.25 * h1))
    ref = 1.5 * g0 - 0.8 * g1 - 0.25
    out = inr.forward(theta, np.zeros((0, 2)), np.array([[x0, x1]]), arch)
    assert abs(out[0] - ref) < 1e-15
    # the same value with omega0 = 1 differs: the factor is applied per layer
    arch1 = configs.INRArch("siren", 2, 0, 0.0, 2, 2, omega0=1.0)
    assert abs(inr.forward(theta, None, np.array([[x0, x1]]), arch1)[0] - ref) > 1e-2


def test_param_counts_of_workloads():
    assert inr.n_params(configs.C1.arch) == 49665
    assert inr.n_params(configs.C2.arch) == 264193
    assert inr.n_params(configs.C3.arch) == 328961
    assert inr.n_params(configs.C4.arch) == 394753


def _fd_vjp(theta, B, X, c, arch, eps=1e-6):
    g = np.zeros_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        g[i] = c @ (inr.forward(tp, B, X, arch) - inr.forward(tm, B, X, arch)) / (2 * eps)
    return g


@pytest.mark.parametrize("arch", [FFN, SIREN, FFN3], ids=["ffn", "siren", "ffn3d"])
def test_vjp_matches_central_differences(arch):
    th, B = _theta(arch, 11)
    rng = np.random.default_rng(12)
    X = rng.uniform(-0.9, 0.9, size=(7, arch.in_dim))
    if arch.kind == "ffn":
        # keep every ReLU pre-activation away from its kink
        for _ in range(100):
            _, _, pre = inr.forward(th, B, X, arch, keep=True)
            bad = np.any(np.abs(np.concatenate(pre, 1)) < 1e-4, axis=1)
            if not bad.any():
                break
            X[bad] = rng.uniform(-0.9, 0.9, size=(bad.sum(), arch.in_dim))
    c = rng.standard_normal(7)
    g = inr.vjp(th, B, X, c, arch)
    fd = _fd_vjp(th, B, X, c, arch)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)


@pytest.mark.parametrize("arch", [FFN, SIREN], ids=["ffn", "siren"])
def test_vjp_matches_torch_autograd(arch):
    th, B = _theta(arch, 21)
    X = np.random.default_rng(22).uniform(-1, 1, size=(13, 2))
    c = np.random.default_rng(23).standard_normal(13)
    t = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    Xt = torch.tensor(X, dtype=torch.float64)
    off, a = 0, None
    if arch.kind == "ffn":
        ph = 2 * math.pi * Xt @ torch.tensor(B, dtype=torch.float64).T
        a = torch.cat([torch.sin(ph), torch.cos(ph)], 1)
    else:
        a = Xt
    dims = inr.layer_dims(arch)
    for li, (fi, fo) in enumerate(dims):
        W = t[off:off + fi * fo].view(fo, fi)
        off += fi * fo
        b = t[off:off + fo]
        off += fo
        a = torch.nn.functional.linear(a, W, b)
        if li < len(dims) - 1:
            a = torch.relu(a) if arch.kind == "ffn" else torch.sin(arch.omega0 * a)
    (a[:, 0] @ torch.tensor(c)).backward()
    assert np.allclose(inr.vjp(th, B, X, c, arch), t.grad.numpy(), rtol=1e-12, atol=1e-13)


def _tiny_problem(arch, seed=0):
    cfg = configs.par2d_problem(8, 6, 11, arch=arch)
    return step.Problem(cfg), cfg


def test_full_sampling_gradient_is_gradient_of_loss():
    # |I| = n: Eq. (2) is grad L(theta) with L = 1/2 ||P E f - y||^2
    for arch in (FFN, SIREN):
        prob, cfg = _tiny_problem(arch)
        th, B = _theta(arch, 31)
        y = np.random.default_rng(32).standard_normal(prob.P.shape[0])

        def L(t):
            return 0.5 * np.sum((prob.P @ prob.E(t, B) - y) ** 2)
        g, _, *_ = step.grad_estimate(prob, th, B, y, prob.fov)
        fd = np.zeros_like(th)
        for i in range(th.size):
            tp, tm = th.copy(), th.copy()
            tp[i] += 1e-6
            tm[i] -= 1e-6
            fd[i] = (L(tp) - L(tm)) / 2e-6
        assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)
        assert prob.n == 52


def test_unbiased_over_all_subsets_and_variance():
    # average of Eq. (2) over all C(52, 2) index pairs equals grad L exactly,
    # and its covariance matches the sampling-without-replacement formula
    prob, cfg = _tiny_problem(FFN)
    th, B = _theta(FFN, 41)
    y = np.random.default_rng(42).standard_normal(prob.P.shape[0])
    g_full, _ = step.full_gradient(prob, th, B, y)
    u = prob.E(th, B)
    v = prob.P.T @ (prob.P @ u - y)
    n, k = prob.n, 2
    # per-point terms a_i = v_i grad f(x_i)
    A = np.stack([inr.vjp(th, B, prob.X[i:i + 1], v[prob.fov[i:i + 1]], FFN)
                  for i in range(n)])
    est = []
    for pair in itertools.combinations(range(n), k):
        g, *_ = step.grad_estimate(prob, th, B, y, prob.fov[list(pair)], v=v)
        est.append(g)
    est = np.array(est)
    assert np.abs(est.mean(0) - g_full).max() <= 1e-12 * np.abs(g_full).max()
    cov = np.cov(est.T, bias=True)
    Abar = A.mean(0)
    S2 = (A - Abar).T @ (A - Abar) / (n - 1)
    ref = n * n * (1 - k / n) / k * S2
    assert np.abs(cov - ref).max() <= 1e-9 * np.abs(ref).max()


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0, 5.0])
    th0 = np.ones(5)
    th, m, v = adam.adam_update(th0, np.zeros(5), np.zeros(5), g, 1, 1e-2)
    ref = th0 - 1e-2 * g / (np.abs(g) + 1e-8)
    assert np.abs(th - ref).max() <= 1e-15


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(5)
    th = rng.standard_normal(17)
    p = torch.nn.Parameter(torch.tensor(th, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(17)
    v = np.zeros(17)
    for t in range(1, 21):
        g = rng.standard_normal(17)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        th, m, v = adam.adam_update(th, m, v, g, t, 3e-3)
    assert np.abs(th - p.detach().numpy()).max() <= 1e-13


def test_seed_average_of_sampled_gradient():
    # mean over 300 PRP draws of Eq. (2) is within 5 sigma of grad L
    from oracle import sampler
    prob, cfg = _tiny_problem(FFN)
    th, B = _theta(FFN, 51)
    y = np.random.default_rng(52).standard_normal(prob.P.shape[0])
    g_full, _ = step.full_gradient(prob, th, B, y)
    v = prob.P.T @ (prob.P @ prob.E(th, B) - y)
    K, k = 300, 8
    est = np.array([step.grad_estimate(
        prob, th, B, y, sampler.sample_indices(prob.fov, k, 777, s), v=v)[0]
        for s in range(K)])
    se = est.std(0, ddof=1) / math.sqrt(K)
    z = np.abs(est.mean(0) - g_full) / np.maximum(se, 1e-300)
    assert np.all(z[se > 0] < 5.0)
