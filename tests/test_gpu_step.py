"""GPU parity of Algorithm 1 + Adam (inr_grad_step) against the oracle."""
import numpy as np
import pytest
import torch

from oracle import adam as oadam
from oracle import sampler as osampler
from oracle import step as ostep
from paper_2604_09884_amd import configs, synth
from tests.gpu_util import dev, host, rel, report, say

pytestmark = pytest.mark.gpu


def _setup(p, dtype, k=None, v_mode=0, loss=0):
    from paper_2604_09884_amd import ops
    k = p.k() if k is None else k
    theta, B = synth.init_inr(p.arch, p.seed_init)
    y = synth.sinogram(p).astype(np.float32)
    m = ops.Model(p.arch, p.dim, p.N, dtype, max_k=k)
    g = ops.Geometry(p)
    th = dev(theta)
    Bd = dev(B.ravel() if B.size else np.zeros(1))
    st = ops.GradStepper(m, g, th, Bd, dev(y.ravel()), k, p.lr, seed=p.seed_sampler,
                         v_mode=v_mode, loss=loss)
    return st, theta, B, y, k


@pytest.mark.parametrize("v_mode", [0, 1], ids=["v_full", "v_at_I"])
def test_single_step_c1(v_mode):
    p = configs.C1
    st, theta, B, y, k = _setup(p, "fp32", v_mode=v_mode)
    prob = ostep.Problem(p)
    st.step(0)
    idx = osampler.sample_indices(prob.fov, k, p.seed_sampler, 0)
    g_ref, L_ref, *_ = ostep.grad_estimate(prob, theta, B, y.astype(np.float64), idx)
    g = host(st.buffer(3, st.model.n_params))
    say("c1 loss", host(st.loss), L_ref, "g rel", rel(g, g_ref))
    report("par2d-128-ffn (C1) step, v %s" % ("full" if v_mode == 0 else "at I"), "fp32", "g",
           rel(g, g_ref), 1e-4)
    report("par2d-128-ffn (C1) step, v %s" % ("full" if v_mode == 0 else "at I"), "fp32",
           "loss", abs(host(st.loss) - L_ref) / L_ref, 1e-5)
    assert abs(host(st.loss) - L_ref) <= 1e-5 * L_ref
    assert rel(g, g_ref) <= 1e-4
    th_ref, _, _ = oadam.adam_update(theta, np.zeros_like(theta), np.zeros_like(theta),
                                     g_ref, 1, p.lr)
    assert np.abs(host(st.theta) - th_ref).max() <= 1e-4 * p.lr + 1e-6


def test_subsampled_step_small_cone():
    p = configs.cone_problem(20, 4, 24, n_ellipses=5, arch=configs.C4.arch.__class__(
        "ffn", 3, 16, 3.0, 128, 2), k_frac=0.1, lr=1e-3)
    st, theta, B, y, k = _setup(p, "fp32")
    prob = ostep.Problem(p)
    st.step(5)
    idx = osampler.sample_indices(prob.fov, k, p.seed_sampler, 5)
    g_ref, L_ref, *_ = ostep.grad_estimate(prob, theta, B, y.reshape(-1).astype(np.float64), idx)
    g = host(st.buffer(3, st.model.n_params))
    say("cone loss", host(st.loss), L_ref, "g rel", rel(g, g_ref))
    report("cone3d-20 step", "fp32", "g", rel(g, g_ref), 1e-4)
    report("cone3d-20 step", "fp32", "loss", abs(host(st.loss) - L_ref) / L_ref, 1e-5)
    assert abs(host(st.loss) - L_ref) <= 1e-5 * L_ref
    assert rel(g, g_ref) <= 1e-4


def test_subsampled_step_small_fan():
    p = configs.fan2d_problem(40, 24, 57, n_ellipses=5, photons=1e5,
                              arch=configs.C6.arch.__class__("ffn", 2, 32, 10.0, 256, 2),
                              k_frac=1.0 / 16, lr=1e-3)
    for dtype, tol in (("fp32", 1e-4), ("bf16", 2e-2)):
        st, theta, B, y, k = _setup(p, dtype)
        prob = ostep.Problem(p)
        st.step(3)
        idx = osampler.sample_indices(prob.fov, k, p.seed_sampler, 3)
        g_ref, L_ref, *_ = ostep.grad_estimate(prob, theta, B, y.reshape(-1).astype(np.float64),
                                               idx)
        g = host(st.buffer(3, st.model.n_params))
        say("fan", dtype, "loss", host(st.loss), L_ref, "g rel", rel(g, g_ref))
        report("fan2d-40 step", dtype, "g", rel(g, g_ref), tol)
        report("fan2d-40 step", dtype, "loss", abs(host(st.loss) - L_ref) / L_ref,
               1e-5 if dtype == "fp32" else tol)
        assert abs(host(st.loss) - L_ref) <= (1e-5 if dtype == "fp32" else tol) * L_ref
        assert rel(g, g_ref) <= tol
        st.close()


def test_c1_fit_final_mse_within_2_percent():
    p = configs.C1
    st, theta, B, y, k = _setup(p, "fp32")
    prob = ostep.Problem(p)
    truth = synth.raster(synth.phantom(p), 2, p.N)
    th, m, v = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    for t in range(p.steps):
        st.step(t)
        idx = osampler.sample_indices(prob.fov, k, p.seed_sampler, t)
        th, m, v, _, _ = ostep.grad_step(prob, th, B, m, v, t + 1, y.astype(np.float64), idx, p.lr)
    torch.cuda.synchronize()
    from paper_2604_09884_amd import ops
    u_gpu = host(ops.inr_eval_grid(st.model, st.theta, st.B))
    mse_gpu = ostep.mse(u_gpu, truth, prob.fov)
    mse_ref = ostep.mse(prob.E(th, B), truth, prob.fov)
    say("c1 20-step MSE gpu", mse_gpu, "oracle", mse_ref)
    report("par2d-128-ffn (C1) 20-step fit", "fp32", "final MSE", abs(mse_gpu - mse_ref) / mse_ref,
           0.02)
    assert abs(mse_gpu - mse_ref) <= 0.02 * mse_ref
