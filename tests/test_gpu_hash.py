"""GPU parity of the hash-encoding INR (E, the Eq. (2) VJP and a whole
step) against the FP64 oracle, FP32 tolerances (1e-4 norm-wise)."""
import numpy as np
import pytest
import torch

from oracle import grid as ogrid
from oracle import inr as oinr
from oracle import sampler as osampler
from oracle import step as ostep
from paper_2604_09884_amd import configs, synth
from tests.gpu_util import dev, host, rel, report, say

pytestmark = pytest.mark.gpu


def _arch(d, W, L, levels, log2, base, top):
    return configs.INRArch("hash", d, 0, 0.0, W, L, hash_levels=levels, hash_feats=2,
                           hash_log2_size=log2, hash_base_res=base, hash_max_res=top)


CASES = [
    ("hash2d-w32", _arch(2, 32, 2, 8, 10, 4, 64), configs.fan2d_problem(45, 16, 67)),
    ("hash3d-w16", _arch(3, 16, 3, 6, 12, 2, 24), configs.cone_problem(20, 6, 24)),
    ("hash2d-w64", _arch(2, 64, 2, 12, 12, 8, 128), configs.par2d_problem(33, 12, 49)),
]


def _away_from_kinks(theta, arch, X, margin):
    _, _, pre = oinr.forward(theta, None, X, arch, keep=True)
    ok = np.ones(X.shape[0], bool)
    for z in pre:
        ok &= np.all(np.abs(z) > margin * np.sqrt(np.mean(z * z)), axis=1)
    return ok


@pytest.mark.parametrize("name,arch,prob", CASES, ids=[c[0] for c in CASES])
def test_hash_eval_and_vjp_match_oracle(name, arch, prob):
    from paper_2604_09884_amd import ops
    say("case", name)
    dim, N = prob.dim, prob.N
    theta, _ = synth.random_theta(arch, 21)
    fov = ogrid.fov_indices(dim, N)
    m = ops.Model(arch, dim, N, "fp32", max_k=fov.size)
    assert m.n_params == arch.n_params == theta.size
    th, Bd = dev(theta), dev(np.zeros(1))
    u = host(ops.inr_eval_grid(m, th, Bd)).ravel()
    u_ref = oinr.eval_grid(theta, None, arch, dim, N, fov, ogrid.coords).ravel()
    say(name, "E rel", rel(u, u_ref))
    assert rel(u, u_ref) <= 1e-4
    assert np.all(u[np.setdiff1d(np.arange(N ** dim), fov)] == 0)
    # point evaluation at a ragged list
    idx = np.sort(np.random.default_rng(22).choice(fov, size=fov.size // 3 + 7, replace=False))
    f = host(ops.inr_eval_points(m, th, Bd, dev(idx, torch.int32)))
    assert rel(f, u_ref[idx]) <= 1e-4
    # Eq. (2) with the cotangent of Algorithm 1 on points away from ReLU kinks
    op = ostep.Problem(prob.with_(arch=arch))
    y = synth.sinogram(prob.with_(n_ellipses=4), noisy=False).ravel()
    v_alg = op.P.T @ (op.P @ op.E(theta, None) - y)
    keep = _away_from_kinks(theta, arch, ogrid.coords(dim, N, fov), 1e-4)
    cand = fov[keep]
    k = max(1, (cand.size * 2) // 3 - 5)
    idx = np.sort(np.random.default_rng(23).choice(cand, size=k, replace=False))
    scale = fov.size / k
    g = host(ops.inr_vjp_subsampled(m, th, Bd, dev(idx, torch.int32), dev(v_alg), scale))
    g_ref = oinr.vjp(theta, None, ogrid.coords(dim, N, idx), scale * v_alg[idx], arch)
    nt = arch.n_table
    say(name, "g rel", rel(g, g_ref), "tables", rel(g[:nt], g_ref[:nt]), "mlp",
        rel(g[nt:], g_ref[nt:]))
    assert rel(g, g_ref) <= 1e-4
    assert rel(g[:nt], g_ref[:nt]) <= 1e-4 and rel(g[nt:], g_ref[nt:]) <= 1e-4
    # entries no point touches are exactly zero, and the result repeats bitwise
    assert np.all(g[:nt][g_ref[:nt] == 0] == 0)
    g2 = host(ops.inr_vjp_subsampled(m, th, Bd, dev(idx, torch.int32), dev(v_alg), scale))
    assert np.array_equal(g, g2)


@pytest.mark.parametrize("v_mode", [0, 1], ids=["v_full", "v_at_I"])
def test_hash_step_matches_oracle(v_mode):
    from paper_2604_09884_amd import ops
    arch = _arch(2, 32, 2, 8, 10, 4, 64)
    p = configs.fan2d_problem(40, 24, 57, arch=arch, k_frac=0.25, n_ellipses=5, lr=1e-3)
    theta, _ = synth.init_inr(arch, p.seed_init)
    y = synth.sinogram(p).astype(np.float32)
    m = ops.Model(arch, 2, p.N, "fp32", max_k=p.k())
    g = ops.Geometry(p)
    st = ops.GradStepper(m, g, dev(theta), dev(np.zeros(1)), dev(y.ravel()), p.k(), p.lr,
                         seed=p.seed_sampler, v_mode=v_mode)
    prob = ostep.Problem(p)
    st.step(2)
    idx = osampler.sample_indices(prob.fov, st.k, p.seed_sampler, 2)
    g_ref, L_ref, *_ = ostep.grad_estimate(prob, theta, None, y.reshape(-1).astype(np.float64),
                                           idx)
    gg = host(st.buffer(3, m.n_params))
    say("hash step loss", float(host(st.loss)), L_ref, "g rel", rel(gg, g_ref))
    assert abs(float(host(st.loss)) - L_ref) <= 1e-5 * L_ref
    assert rel(gg, g_ref) <= 1e-4
    st.close()


def test_hash_full_size_sampled():
    # the 512^2 hash workload's model: E at sampled FOV points and the VJP
    # of a sampled index set, against the oracle point by point
    from paper_2604_09884_amd import ops
    p = configs.C7
    arch, N = p.arch, p.N
    theta, _ = synth.random_theta(arch, 31)
    fov = ogrid.fov_indices(2, N)
    m = ops.Model(arch, 2, N, "fp32", max_k=p.k())
    th, Bd = dev(theta), dev(np.zeros(1))
    u = host(ops.inr_eval_grid(m, th, Bd)).ravel()
    pts = np.unique(np.concatenate([fov[np.random.default_rng(32).choice(fov.size, 4000)],
                                    [fov[0], fov[-1]]]))
    e = rel(u[pts], oinr.forward(theta, None, ogrid.coords(2, N, pts), arch))
    say("C7 E sampled rel", e)
    report("fan2d-512-hash (C7)", "fp32", "E, sampled points", e, 1e-4)
    assert e <= 1e-4
    keep = _away_from_kinks(theta, arch, ogrid.coords(2, N, pts), 1e-4)
    idx = pts[keep][:2000]
    v = np.random.default_rng(33).standard_normal(idx.size)
    g = host(ops.inr_vjp_subsampled(m, th, Bd, dev(idx, torch.int32), dev(v), 3.0,
                                    v_compact=True))
    g_ref = oinr.vjp(theta, None, ogrid.coords(2, N, idx), 3.0 * v, arch)
    say("C7 g rel", rel(g, g_ref))
    report("fan2d-512-hash (C7)", "fp32", "g", rel(g, g_ref), 1e-4)
    assert rel(g, g_ref) <= 1e-4


def test_hash_full_size_table_gradient_at_full_k():
    # |I| = n/16 = 12,868 points of the 512^2 hash workload: 823,552
    # table-gradient contributions, sorted on 23-bit keys in three passes
    # over 403 tiles; against the oracle, and bitwise repeatable
    from paper_2604_09884_amd import ops
    p = configs.C7
    arch, N = p.arch, p.N
    theta, _ = synth.random_theta(arch, 34)
    fov = ogrid.fov_indices(2, N)
    k = p.k()
    m = ops.Model(arch, 2, N, "fp32", max_k=k)
    th, Bd = dev(theta), dev(np.zeros(1))
    cand = np.sort(np.random.default_rng(35).choice(fov, 2 * k, replace=False))
    keep = _away_from_kinks(theta, arch, ogrid.coords(2, N, cand), 1e-4)
    idx = cand[keep][:k]
    assert idx.size == k
    v = np.random.default_rng(36).standard_normal(k)
    g = host(ops.inr_vjp_subsampled(m, th, Bd, dev(idx, torch.int32), dev(v), 16.0,
                                    v_compact=True))
    g2 = host(ops.inr_vjp_subsampled(m, th, Bd, dev(idx, torch.int32), dev(v), 16.0,
                                     v_compact=True))
    assert np.array_equal(g, g2)
    g_ref = oinr.vjp(theta, None, ogrid.coords(2, N, idx), 16.0 * v, arch)
    e = rel(g, g_ref)
    et = rel(g[:arch.n_table], g_ref[:arch.n_table])
    say("C7 full-k g rel", e, "table part", et)
    report("fan2d-512-hash (C7)", "fp32", "g at |I| = 12,868", e, 1e-4)
    assert e <= 1e-4 and et <= 1e-4


def test_hash_single_point_and_all_hashed_levels():
    # k = 1, and a 3D model whose every level is hashed (T = 2^6 < (N_0+1)^3)
    from paper_2604_09884_amd import ops
    arch = _arch(3, 16, 1, 3, 6, 4, 9)
    N = 11
    theta, _ = synth.random_theta(arch, 41)
    fov = ogrid.fov_indices(3, N)
    m = ops.Model(arch, 3, N, "fp32", max_k=5)
    th, Bd = dev(theta), dev(np.zeros(1))
    u = host(ops.inr_eval_grid(m, th, Bd)).ravel()
    assert rel(u, oinr.eval_grid(theta, None, arch, 3, N, fov, ogrid.coords).ravel()) <= 1e-4
    idx = fov[[fov.size // 2]]
    g = host(ops.inr_vjp_subsampled(m, th, Bd, dev(idx, torch.int32), dev(np.array([0.7])), 2.0,
                                    v_compact=True))
    g_ref = oinr.vjp(theta, None, ogrid.coords(3, N, idx), np.array([1.4]), arch)
    assert rel(g, g_ref) <= 1e-4
    assert np.count_nonzero(g[:arch.n_table]) <= 3 * 8 * 2
