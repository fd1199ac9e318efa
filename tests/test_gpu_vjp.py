"""GPU parity of the subsampled Jacobian-transpose product (Eq. (2)) at
the chunked shapes the 501^3 step runs, and of the autograd route through
the virtual loss of Eq. (3) (Algorithm 1, steps 4-5), against the FP64
oracle."""
import numpy as np
import pytest
import torch

from oracle import grid as ogrid
from oracle import inr as oinr
from oracle import sampler as osampler
from paper_2604_09884_amd import configs, synth
from tests.gpu_util import dev, host, rel, report, say

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng
CHUNK = 262144  # points per VJP scratch chunk in the library


def _ops():
    from paper_2604_09884_amd import ops
    return ops


def _away_from_kinks(theta, B, arch, X, margin, block=50000):
    """Rows of X whose ReLU pre-activations all lie farther than
    margin * rms from 0 (no decision can flip between FP64 and FP32)."""
    ok = np.ones(X.shape[0], bool)
    for a in range(0, X.shape[0], block):
        _, _, pre = oinr.forward(theta, B, X[a:a + block], arch, keep=True)
        for z in pre:
            ok[a:a + block] &= np.all(np.abs(z) > margin * np.sqrt(np.mean(z * z)), axis=1)
    return ok


def _oracle_vjp(theta, B, X, cot, arch, block=65536):
    """Eq. (2)'s sum by the oracle, over blocks of points (the sum is linear
    in the points; float64 throughout)."""
    g = np.zeros(theta.size)
    for a in range(0, X.shape[0], block):
        g += oinr.vjp(theta, B, X[a:a + block], cot[a:a + block], arch)
    return g


def _smooth_field(X, seed):
    """A smooth cotangent field over the points (a sum of Gaussians), the
    kind of v that P^T of a residual produces."""
    rng = RNG(seed)
    v = np.zeros(X.shape[0])
    for _ in range(6):
        c = rng.uniform(-0.7, 0.7, X.shape[1])
        v += rng.uniform(-1, 1) * np.exp(-np.sum((X - c) ** 2, 1) / (2 * 0.3 ** 2))
    return v


def test_vjp_fp32_across_chunks_c4_arch():
    # k above one chunk: the dW partials accumulate across chunks
    ops = _ops()
    arch = configs.C4.arch
    N = 96
    fov = ogrid.fov_indices(3, N)
    theta, B = synth.random_theta(arch, 17)
    cand = np.sort(RNG(18).choice(fov, size=400000, replace=False))
    idx = cand[_away_from_kinks(theta, B, arch, ogrid.coords(3, N, cand), 2e-4)]
    k = idx.size
    say("fp32 multi-chunk k", k, "chunks", -(-k // CHUNK))
    assert k > CHUNK + 1000
    m = ops.Model(arch, 3, N, "fp32", max_k=k)
    v = RNG(19).standard_normal(k)
    g = host(ops.inr_vjp_subsampled(m, dev(theta), dev(B.ravel()), dev(idx, torch.int32),
                                    dev(v), 1.5, v_compact=True))
    g_ref = _oracle_vjp(theta, B, ogrid.coords(3, N, idx), 1.5 * v, arch)
    e = rel(g, g_ref)
    say("fp32 multi-chunk g rel", e)
    report("ffn 3->512+5x256, %d points (2 chunks)" % k, "fp32", "g (VJP)", e, 1e-4)
    assert e <= 1e-4
    # linearity across chunks: the sum over I equals the sum of the halves
    h = k // 2
    ga = host(ops.inr_vjp_subsampled(m, dev(theta), dev(B.ravel()), dev(idx[:h], torch.int32),
                                     dev(v[:h]), 1.5, v_compact=True))
    gb = host(ops.inr_vjp_subsampled(m, dev(theta), dev(B.ravel()), dev(idx[h:], torch.int32),
                                     dev(v[h:]), 1.5, v_compact=True))
    assert rel(ga + gb, g) <= 1e-5


def test_vjp_bf16_width256_across_chunks():
    # the BF16 width-256 kernels (forward recompute + backward per tile, then
    # the dW contraction with its split-K partials accumulated over chunks)
    ops = _ops()
    arch = configs.C4.arch
    N = 112
    fov = ogrid.fov_indices(3, N)
    theta, B = synth.random_theta(arch, 27)
    idx = np.sort(RNG(28).choice(fov, size=3 * CHUNK + 12345, replace=False))
    k = idx.size
    X = ogrid.coords(3, N, idx)
    v = _smooth_field(X, 29)
    m = ops.Model(arch, 3, N, "bf16", max_k=k)
    g = host(ops.inr_vjp_subsampled(m, dev(theta), dev(B.ravel()), dev(idx, torch.int32),
                                    dev(v), 0.75, v_compact=True))
    g_ref = _oracle_vjp(theta, B, X, 0.75 * v, arch)
    e = rel(g, g_ref)
    say("bf16 width-256 g rel over %d chunks (k %d)" % (-(-k // CHUNK), k), e)
    report("ffn 3->512+5x256, %d points (4 chunks)" % k, "bf16", "g (VJP)", e, 2e-2)
    assert e <= 2e-2
    # the last, ragged chunk alone against its own oracle sum
    tail = slice(3 * CHUNK, k)
    gt = host(ops.inr_vjp_subsampled(m, dev(theta), dev(B.ravel()),
                                     dev(idx[tail], torch.int32), dev(v[tail]), 0.75,
                                     v_compact=True))
    et = rel(gt, _oracle_vjp(theta, B, X[tail], 0.75 * v[tail], arch))
    say("bf16 ragged tail chunk g rel", et)
    assert et <= 2e-2


def test_vjp_bf16_width128_across_chunks():
    # the BF16 width-128 FFN of the serving mix's 3D requests (64 frequencies,
    # 3 x 128): two column tiles a wave in the recompute, and the 128 x 128
    # dW tiles with their split-K partials accumulated over three chunks
    from paper_2604_09884_amd import configs as cfg
    ops = _ops()
    arch = cfg.serving_mix(64)[1].arch
    assert arch.kind == "ffn" and arch.width == 128
    N = 96
    fov = ogrid.fov_indices(3, N)
    theta, B = synth.random_theta(arch, 37)
    idx = np.sort(RNG(38).choice(fov, size=2 * CHUNK + 4321, replace=False))
    k = idx.size
    X = ogrid.coords(3, N, idx)
    v = _smooth_field(X, 39)
    m = ops.Model(arch, 3, N, "bf16", max_k=k)
    g = host(ops.inr_vjp_subsampled(m, dev(theta), dev(B.ravel()), dev(idx, torch.int32),
                                    dev(v), 1.5, v_compact=True))
    g_ref = _oracle_vjp(theta, B, X, 1.5 * v, arch)
    e = rel(g, g_ref)
    say("bf16 width-128 g rel over %d chunks (k %d)" % (-(-k // CHUNK), k), e)
    report("ffn 3->128+3x128, %d points (3 chunks)" % k, "bf16", "g (VJP)", e, 2e-2)
    assert e <= 2e-2
    # every layer's weight and bias blocks on their own (a dW tile that
    # missed a block of rows or columns would show here)
    off = arch.n_table
    for fi, fo in arch.layer_dims():
        for n in (fi * fo, fo):
            eb = rel(g[off:off + n], g_ref[off:off + n])
            say("  block of %d: rel %.3e" % (n, eb))
            assert eb <= 5e-2
            off += n
    assert off == g.size


def test_vjp_at_the_501_cube_index_set():
    # the 987,757-point I the 501^3 step draws at step 0 (four chunks),
    # with a smooth cotangent and the step's scale n/k, BF16 as benchmarked
    ops = _ops()
    p = configs.C4
    theta, B = synth.init_inr(p.arch, p.seed_init)
    m = ops.Model(p.arch, 3, p.N, "bf16", max_k=p.k())
    n, k = m.n_fov, p.k(m.n_fov)
    idx_d = ops.sample(m, p.seed_sampler, 0, k)
    idx = host(idx_d).astype(np.int64)
    fov = ogrid.fov_indices(3, p.N)
    assert idx.size == 987757 and np.array_equal(idx, osampler.sample_indices(fov, k,
                                                                              p.seed_sampler, 0))
    X = ogrid.coords(3, p.N, idx)
    v = _smooth_field(X, 31)
    scale = n / k
    g = host(ops.inr_vjp_subsampled(m, dev(theta), dev(B.ravel()), idx_d, dev(v), scale,
                                    v_compact=True))
    g_ref = _oracle_vjp(theta, B, X, scale * v, p.arch, block=100000)
    e = rel(g, g_ref)
    say("501^3 I: k %d, g rel %.3e (BF16, %d chunks)" % (k, e, -(-k // CHUNK)))
    report("cone3d-501 (C4) index set, 987,757 points", "bf16", "g (VJP)", e, 2e-2)
    assert e <= 2e-2


@pytest.mark.parametrize("case", ["c1_full", "c1_sampled", "bf16_256"])
def test_inr_function_virtual_loss_backward(case):
    # Eq. (3): L~ = (n/|I|) sum_{i in I} v_i f_theta(x_i) with v the
    # cotangent Algorithm 1 forms, P^T (P E f - y); its gradient by torch
    # autograd through INRFunction (forward on the matrix cores, backward the
    # hand-written VJP) equals the oracle's exact Eq. (2) sum
    from oracle import step as ostep
    ops = _ops()
    if case == "bf16_256":
        p = configs.fan2d_problem(48, 24, 71, arch=configs.C6.arch)
        dtype, tol = "bf16", 2e-2
    else:
        p = configs.C1
        dtype, tol = "fp32", 1e-4
    prob = ostep.Problem(p)
    fov, n = prob.fov, prob.n
    theta, B = synth.random_theta(p.arch, 41)
    y = synth.sinogram(p.with_(n_ellipses=4), noisy=False).ravel()
    v_alg = prob.P.T @ (prob.P @ prob.E(theta, B) - y)
    if case == "c1_sampled":
        idx = np.sort(RNG(42).choice(fov, size=n // 7, replace=False))
    else:
        idx = fov
    X = ogrid.coords(p.dim, p.N, idx)
    v = v_alg[idx]
    k = idx.size
    m = ops.Model(p.arch, p.dim, p.N, dtype, max_k=k)
    th = dev(theta).requires_grad_(True)
    Bd = dev(B.ravel())
    idx_d = dev(idx, torch.int32)
    f = ops.INRFunction.apply(th, Bd, idx_d, m)
    f_ref = oinr.forward(theta, B, X, p.arch)
    ef = rel(host(f), f_ref)
    Lv = (n / k) * torch.sum(dev(v) * f)
    Lv.backward()
    g = host(th.grad)
    g_ref = oinr.vjp(theta, B, X, (n / k) * v, p.arch)
    eg = rel(g, g_ref)
    say("INRFunction %s: |I| %d of n %d, f rel %.3e, g rel %.3e" % (case, k, n, ef, eg))
    report("INRFunction %s" % case, dtype, "g (virtual-loss backward)", eg, tol)
    assert ef <= tol and eg <= tol
