"""Benchmark: memory-efficient INR gradient steps per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c4]
                    [--v-mode full|at_i] [--mlp-dtype bf16|fp32] [--no-cpu]

One step is one pass of the whole hot path (Algorithm 1 + Adam) on the
501^3, 20-view, 768^2-detector cone-beam workload: grid evaluation of the
FFN INR (3 -> 512 Fourier features + 5 x 256 ReLU -> 1) on all 98,775,657
FOV voxels, Joseph projection, LS residual, matched adjoint, 1% index
sample, subsampled VJP, Adam.  Inputs are seeded synthetic data
(random-ellipsoid phantom, closed-form chord data, Poisson noise at 1e5
photons) resident on the GPU before timing starts.

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (the grid-evaluation GEMM chain, timed with HIP events on its own
stream) and the FP64 oracle timed on a bounded sample on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2.5e15, "fp32": 157.3e12}   # dense MFMA FLOP/s, MI355X


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c4")
    ap.add_argument("--v-mode", default="full", choices=["full", "at_i"])
    ap.add_argument("--loss", default="ls", choices=["ls", "fls"],
                    help="data term: least squares, or the ramp-filtered FLS loss")
    ap.add_argument("--mlp-dtype", default=None, choices=[None, "bf16", "fp32"])
    ap.add_argument("--subsets", type=int, default=1,
                    help="ordered subsets over views: step t takes the loss over views j "
                         "with j mod S == t mod S")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve", type=int, default=0, metavar="R",
                    help="measure serving instead: a Poisson stream of R requests of the "
                         "mixed 2D/3D serving mix (prints its own JSON line)")
    ap.add_argument("--serve-steps", type=int, default=500)
    ap.add_argument("--serve-rate", type=float, default=2.0, help="arrivals per second")
    ap.add_argument("--serve-slots", type=int, default=8,
                    help="requests resident and stepping at once")
    ap.add_argument("--no-stream", action="store_true",
                    help="with --serve-compare: run only the comparison, not the stream")
    ap.add_argument("--serve-compare", type=int, default=0, metavar="Q",
                    help="with --serve: also the first Q requests in FP32 one at a time "
                         "against BF16 served together, with every request's final image MSE")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy before the steps (a "
                         "reference for hardware byte counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(p, target_s):
    """The FP64 oracle on a bounded sample of one step, scaled to a whole
    step: E on a sample of FOV points, P and P^T on a sample of rays, the
    VJP on a sample of the index set, the sampler on a sample of draws, Adam
    on all parameters."""
    from threadpoolctl import threadpool_info

    from oracle import adam as oadam
    from oracle import geometry as ogeo
    from oracle import grid as ogrid
    from oracle import inr as oinr
    from oracle import joseph
    from oracle import sampler as osampler
    from paper_2604_09884_amd import synth

    rng = np.random.default_rng(0)
    theta, B = synth.init_inr(p.arch, p.seed_init)
    n = p.n_fov()
    k = p.k(n)
    m = p.n_rays
    fov2 = ogrid.fov_indices(2, p.N)
    budget = target_s / 5.0

    def timed(fn):
        t = time.perf_counter()
        fn()
        return time.perf_counter() - t

    # E: oracle forward on S points (grow S until ~budget)
    S = 2048
    nz = p.N if p.dim == 3 else 1
    while True:
        pts = fov2[rng.choice(fov2.size, size=S)] + rng.integers(0, nz, S) * p.N * p.N
        X = ogrid.coords(p.dim, p.N, pts)
        t_e = timed(lambda: oinr.forward(theta, B, X, p.arch))
        if t_e > budget / 2 or S >= min(1 << 18, n):
            break
        S = min(2 * S, n)
    per_E = t_e / S * n
    # P and P^T on R rays drawn from four random views (and, in 3-D, eight
    # random detector rows of them)
    views = np.sort(rng.choice(p.n_views, size=min(4, p.n_views), replace=False))
    if p.dim == 3:
        rows = np.sort(rng.choice(p.n_v, size=min(8, p.n_v), replace=False))
        p0, d = ogeo.cone3d_rays(p.n_views, p.n_u, p.n_v, p.du, p.dv, p.dso, p.dod,
                                 p.view_span, views=views, rows=rows)
    else:
        p0, d = ogeo.problem_rays(p, views=views)
    R = min(1024, p0.shape[0])
    sel = rng.choice(p0.shape[0], size=R, replace=False)
    t0 = time.perf_counter()
    A = joseph.system_matrix(p.N, p.dim, p0[sel], d[sel])
    t_build = time.perf_counter() - t0
    vol = np.ones(p.N ** p.dim)
    t_p = t_build + timed(lambda: A @ vol)
    r = rng.standard_normal(R)
    t_pt = t_build + timed(lambda: A.T @ r)
    del vol
    per_P = t_p / R * m
    per_PT = t_pt / R * m
    # VJP on Q sampled points
    Q = 1024
    Xq = ogrid.coords(p.dim, p.N, fov2[rng.choice(fov2.size, size=Q)]
                      + (nz // 2) * p.N * p.N)
    t_v = timed(lambda: oinr.vjp(theta, B, Xq, rng.standard_normal(Q), p.arch))
    per_V = t_v / Q * k
    # sampler on D draws
    D = 2000
    t_s = timed(lambda: osampler.sample_ranks(n, D, 1, 0))
    per_S = t_s / D * k
    # Adam on all parameters
    t_a = timed(lambda: oadam.adam_update(theta, np.zeros_like(theta), np.zeros_like(theta),
                                          theta, 1, 1e-3))
    total = per_E + per_P + per_PT + per_V + per_S + t_a
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {
        "value": 1.0 / total, "unit": "steps/s", "cores": int(threads), "kind": "oracle",
        "sample": ("FP64 oracle on a bounded sample scaled to one full step: E on %d FOV "
                   "points (x%.0f), P and P^T on %d rays of 4 random views%s (x%.0f), VJP on %d samples "
                   "(x%.0f), sampler on %d draws, Adam on all %d parameters; "
                   "est. %.1f s per step (E %.1f s, P %.1f s, P^T %.1f s, VJP %.1f s)"
                   % (S, n / S, R, " and 8 random rows" if p.dim == 3 else "", m / R, Q,
                      k / Q, D, theta.size, total, per_E, per_P,
                      per_PT, per_V)),
        "host_cpus": os.cpu_count(),
    }


PROFILE_SOURCES = {
    "mlp": os.path.join("paper_2604_09884_amd", "csrc", "mlp.hip"),
    "cone": os.path.join("paper_2604_09884_amd", "csrc", "cone.hip"),
    "projector": os.path.join("paper_2604_09884_amd", "csrc", "projector.hip"),
}


def profile_figures(name):
    """Per-kernel figures (HBM bytes per launch from FETCH_SIZE / WRITE_SIZE,
    VALU busy and matrix-core utilisation) from the JSON block of a committed
    counter summary under profiles/, keeping only the kernels whose source
    file still hashes to the value recorded with the counters."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", name)).read()
    except OSError:
        return {}
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return {}
    data = json.loads(m.group(1))
    shas = {}
    for key, rel in PROFILE_SOURCES.items():
        try:
            shas[key] = hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()
        except OSError:
            shas[key] = None
    out = {}
    for kernel, rec in data.get("kernels", {}).items():
        src = rec.get("source")
        if src in shas and rec.get("sha256") == shas[src]:
            out[kernel] = rec
    return out


def _fig(figs, kernels, field):
    """Sum (bytes) of a field over kernels, or None if any is missing."""
    vals = [figs.get(k, {}).get(field) for k in kernels]
    return None if any(v is None for v in vals) else sum(vals)


def _sinograms(probs):
    """Seeded synthetic data of every request (closed-form chords, host work
    done before any timing; large sinograms spread their views over threads)."""
    from paper_2604_09884_amd import synth
    out = []
    t0 = time.time()
    for i, p in enumerate(probs):
        out.append(synth.sinogram(p).astype(np.float32))
        if i % 8 == 7 or i == len(probs) - 1:
            log("  sinograms %d/%d (%.1f s)" % (i + 1, len(probs), time.time() - t0))
    return out


def _fov_mask(dim, N):
    c = -1.0 + (np.arange(N) + 0.5) * (2.0 / N)
    disc = (c[None, :] ** 2 + c[:, None] ** 2) <= 1.0
    return disc if dim == 2 else np.broadcast_to(disc, (N, N, N))


def _final_mse(p, theta):
    """Final-image MSE over the FOV against the rasterised phantom, with
    the INR evaluated on the GPU in FP32."""
    import torch

    from paper_2604_09884_amd import ops, synth
    m = ops.Model(p.arch, p.dim, p.N, "fp32", max_k=1)
    th = torch.tensor(theta, dtype=torch.float32, device="cuda")
    _, B = synth.init_inr(p.arch, p.seed_init)
    Bd = torch.tensor(B.ravel() if B.size else np.zeros(1), dtype=torch.float32, device="cuda")
    u = ops.inr_eval_grid(m, th, Bd).cpu().numpy().reshape([p.N] * p.dim)
    ref = synth.raster(synth.phantom(p), p.dim, p.N)
    msk = _fov_mask(p.dim, p.N)
    m.close()
    return float(np.mean((u[msk] - ref[msk]) ** 2))


def _serve(probs, ys, arrivals, dtype, n_slots, depth=2):
    """Runs the requests through one server (arrival times on its clock;
    None: all at once) and returns (server, request ids)."""
    import torch

    from paper_2604_09884_amd.serve import Request, Server
    srv = Server(n_slots=n_slots, depth=depth)
    ids = [srv.submit(Request(problem=p, y=y, steps=p.steps, mlp_dtype=dtype),
                      arrival=None if arrivals is None else float(t))
           for p, y, t in zip(probs, ys, arrivals if arrivals is not None else [0] * len(probs))]
    torch.cuda.synchronize()
    srv.t0 = time.perf_counter()
    for i in ids:  # arrival times count from the start of the run
        if arrivals is None:
            srv.slots[i].t_arrive = 0.0

    def progress(sv):
        m = sv.metrics()
        log("  t %.0f s: %d done, %d active, %d queued, %d steps"
            % (sv.now(), m["done"], len(sv.active()), len(sv.queue), m["steps"]))
    srv.run(progress=progress)
    torch.cuda.synchronize()
    return srv, ids


def serve_bench(a):
    """The serving workload: a seeded Poisson stream of requests (mean rate
    --serve-rate per second) from the mixed 2D/3D request mix, each a
    --serve-steps-step fit, served with continuous batching in BF16.
    Reports time-to-reconstruction percentiles (completion minus arrival),
    aggregate steps/s and makespan.  With --serve-compare Q, the first Q
    requests are also run in FP32 one at a time (back to back) and in BF16
    served together, with each request's final image MSE in both forms."""
    import torch

    from paper_2604_09884_amd import configs
    from paper_2604_09884_amd.serve import DONE, poisson_arrivals

    probs = configs.serving_mix(a.serve, steps=a.serve_steps)
    arrivals = poisson_arrivals(len(probs), a.serve_rate, 5005)
    t0 = time.time()
    ys = _sinograms(probs)
    log("serving stream: %d requests over %.1f s of arrivals; sinograms in %.1f s"
        % (len(probs), arrivals[-1], time.time() - t0))
    torch.cuda.set_device(0)
    # warm-up: one request of each kind for one step (kernel loading)
    seen = set()
    warm = []
    for p, y in zip(probs, ys):
        key = (p.dim, p.arch.kind)
        if key not in seen:
            seen.add(key)
            warm.append((p.with_(steps=1), y))
    _serve([w[0] for w in warm], [w[1] for w in warm], None, "bf16", a.serve_slots)
    if a.no_stream:
        m = {k_: None for k_ in ("latency_s_p50", "latency_s_p95", "latency_s_p99",
                                 "latency_s_max", "queue_wait_s_p50", "queue_wait_s_p99",
                                 "steps_per_s", "makespan_s", "done", "failed")}
    else:
        srv, ids = _serve(probs, ys, arrivals, "bf16", a.serve_slots)
        m = srv.metrics()
        bad = [srv.status(i).error for i in ids if srv.status(i).state != DONE]
        log("served: %s%s" % ({k: round(v, 3) if isinstance(v, float) else v
                               for k, v in m.items()}, " failures %s" % bad if bad else ""))
    out = {
        "metric": "p99 recon latency (served mixed 2D/3D stream)",
        "value": m["latency_s_p99"], "unit": "s", "higher_is_better": False, "n_gpus": 1,
        "latency_s": {"p50": m["latency_s_p50"], "p95": m["latency_s_p95"],
                      "p99": m["latency_s_p99"], "max": m["latency_s_max"]},
        "queue_wait_s": {"p50": m["queue_wait_s_p50"], "p99": m["queue_wait_s_p99"]},
        "steps_per_s": m["steps_per_s"], "makespan_s": m["makespan_s"],
        "requests": len(probs), "done": m["done"], "failed": m["failed"],
        "steps_per_request": a.serve_steps, "arrival_rate_per_s": a.serve_rate,
        "slots": a.serve_slots, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "C5 serving stream (Poisson arrivals seed 5005, mix seed 5005)",
                   "mix": [p.name + ":" + p.arch.kind for p in probs]},
    }
    if a.serve_compare:
        q = min(a.serve_compare, len(probs))
        sub, suby = probs[:q], ys[:q]
        t = time.perf_counter()
        alone = []
        for p, y in zip(sub, suby):
            s1, i1 = _serve([p], [y], None, "fp32", 1)
            assert s1.status(i1[0]).state == DONE, s1.status(i1[0]).error
            alone.append(s1.status(i1[0]).theta)
            log("FP32 alone: %s done" % p.name)
        t_fp32 = time.perf_counter() - t
        t = time.perf_counter()
        s2, i2 = _serve(sub, suby, None, "bf16", a.serve_slots)
        t_bf16 = time.perf_counter() - t
        mse32 = [_final_mse(p, th) for p, th in zip(sub, alone)]
        mse16 = [_final_mse(p, s2.status(i).theta) for p, i in zip(sub, i2)]
        rel = [abs(b - f) / f for f, b in zip(mse32, mse16)]
        steps = sum(p.steps for p in sub)
        out["compare"] = {
            "requests": q, "steps_per_request": a.serve_steps,
            "fp32_one_at_a_time_steps_per_s": steps / t_fp32,
            "bf16_served_steps_per_s": steps / t_bf16, "speedup": t_fp32 / t_bf16,
            "final_mse_fp32_alone": mse32, "final_mse_bf16_served": mse16,
            "max_rel_mse_difference": max(rel), "median_rel_mse_difference": float(np.median(rel)),
            "mix": [p.name + ":" + p.arch.kind for p in sub],
        }
        log("compare: FP32 alone %.1f steps/s, BF16 served %.1f steps/s, max rel MSE diff %.3g"
            % (steps / t_fp32, steps / t_bf16, max(rel)))
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % a.gpus, flush=True)
        sys.exit(2)
    if a.serve:
        serve_bench(a)
        return
    import torch

    from paper_2604_09884_amd import configs, lib as L, ops, synth

    p = configs.CONFIGS[a.config]
    dtype = a.mlp_dtype or p.mlp_dtype
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    t0 = time.time()
    theta, B = synth.init_inr(p.arch, p.seed_init)
    y = synth.sinogram(p).astype(np.float32)
    log("inputs synthesised in %.1f s" % (time.time() - t0))
    free0, total_mem = torch.cuda.mem_get_info()
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    Bd = torch.tensor(B.ravel() if B.size else np.zeros(1), dtype=torch.float32, device=dev)
    yd = torch.tensor(y.ravel(), device=dev)
    model = ops.Model(p.arch, p.dim, p.N, dtype, max_k=p.k())
    geom = ops.Geometry(p)
    k = p.k(model.n_fov)
    v_mode = L.INRCT_V_FULL if a.v_mode == "full" else L.INRCT_V_AT_I
    loss_kind = L.INRCT_FLS if a.loss == "fls" else L.INRCT_LS
    st = ops.GradStepper(model, geom, th, Bd, yd, k, p.lr, seed=p.seed_sampler, v_mode=v_mode,
                         loss=loss_kind)
    stepper = ops.OrderedSubsets(st, a.subsets) if a.subsets > 1 else st
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    log("n_fov %d, k %d, params %d, device memory in use %.2f GB"
        % (model.n_fov, k, model.n_params, (free0 - free1) / 1e9))

    if a.calib_copy:
        src = torch.ones(1 << 28, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for t in range(a.warmup):
        stepper.step(t)
    torch.cuda.synchronize()
    log("warmup done (%d steps), loss %.6g" % (a.warmup, float(st.loss)))
    st.enable_timing(max(1, a.steps))
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for t in range(a.steps):
        stepper.step(a.warmup + t)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    stages = st.stage_ms()
    free2, _ = torch.cuda.mem_get_info()
    ms_step = wall * 1e3 / a.steps
    loss = float(st.loss)
    log("timed %d steps: %.2f ms/step, loss %.6g, stages %s"
        % (a.steps, ms_step, loss, {k_: round(v / a.steps, 3) for k_, v in stages.items()}))

    # the same steps with v formed only at the sampled points (the entries
    # Eq. (2) consumes; the same g up to summation order), from the same
    # starting parameters, reported beside the literal full-grid v
    alt = None
    if a.v_mode == "full" and a.subsets == 1:
        th2 = torch.tensor(theta, dtype=torch.float32, device=dev)
        st2 = ops.GradStepper(model, geom, th2, Bd, yd, k, p.lr, seed=p.seed_sampler,
                              v_mode=L.INRCT_V_AT_I, loss=loss_kind)
        for t in range(a.warmup):
            st2.step(t)
        st2.enable_timing(max(1, a.steps))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for t in range(a.steps):
            st2.step(a.warmup + t)
        torch.cuda.synchronize()
        ms2 = (time.perf_counter() - t2) * 1e3 / a.steps
        st2_stages = st2.stage_ms()
        alt = {"v_mode": "at_i", "value": 1e3 / ms2, "ms_per_step": ms2,
               "backproject_ms": st2_stages["backproject"] / a.steps,
               "loss_last": float(st2.loss)}
        log("v at I: %.2f ms/step (P^T at I %.3f ms)" % (ms2, alt["backproject_ms"]))
        st2.close()

    figs = {}
    if a.config == "c4" and dtype == "bf16" and a.subsets == 1:
        figs.update(profile_figures("step_c4_hbm_traffic.md"))
        util = profile_figures("step_c4_utilization.md")
        for k_, rec in util.items():
            figs.setdefault(k_, {}).update(rec)
    e_kernel = ("k_hash_eval" if p.arch.kind == "hash"
                else "k_eval_grid" if dtype == "fp32"
                else "k_eval_lds_w<%d>" % (1 if p.arch.kind == "ffn" else 2))
    traffic = _fig(figs, [e_kernel], "traffic_bytes")
    flop_per_point = p.arch.flops_forward()
    if p.arch.kind == "hash":  # plus the interpolation: 2^d weights x 2 features per level
        flop_per_point += p.arch.hash_levels * (1 << p.dim) * 2 * 2
    e_ms = stages["eval_grid"] / a.steps
    achieved = model.n_fov * flop_per_point / (e_ms * 1e-3)
    hashed = p.arch.kind == "hash"
    # a gather-latency kernel in FP32 vector arithmetic without packed
    # instructions: peak 256 CUs x 64 lanes x 2 FLOP x 2.4 GHz = 78.6 TFLOP/s
    peak = 78.6e12 if hashed else PEAK[dtype]
    roofline = {"bound": "alu" if hashed else "mfma",
                "kernel": e_kernel + " (grid evaluation E)",
                "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE, WRITE_SIZE, copy-calibrated; "
                                "profiles/step_c4_hbm_traffic.md)",
                "per_unit": "%d FLOP per FOV point x %d points per launch"
                            % (flop_per_point, model.n_fov),
                "avg_launch_ms": e_ms}
    mfma_util = _fig(figs, [e_kernel], "mfma_util")
    if mfma_util is not None:
        roofline["mfma_busy_counter"] = mfma_util
    stage_roofs = None
    if p.dim == 3:
        n_grid = p.N ** 3
        m_rays = geom.n_rays
        p_ms = stages["project"] / a.steps
        pt_ms = stages["backproject"] / a.steps
        v_ms = stages["vjp"] / a.steps
        p_bytes = p.n_views * model.n_fov * 4 + m_rays * 4
        pt_bytes = m_rays * 4 + n_grid * 4
        # the P stage: the plane-wise transpose, then both tile sets through
        # the row kernel (figures per step, summed over launches)
        p_kernels = ["k_transpose2d", "k_cone_fwd_lds<true>"]
        pt_kernels = ["k_cone_prescale", "k_cone_bp_lds<true>"]
        p_traffic = _fig(figs, p_kernels, "traffic_bytes")
        pt_traffic = _fig(figs, pt_kernels, "traffic_bytes")
        vjp_flop = p.arch.flops_vjp() * k  # forward recompute + dW + delta, per sample
        stage_roofs = {
            "P": {"kernels": p_kernels, "ms": p_ms, "bound": "alu",
                  "hbm_alg_bytes": p_bytes,
                  "hbm_alg_note": "view-major model: every view reads the FOV volume once "
                                  "(%d x %d x 4 B) and writes its rays (%d x 4 B)"
                                  % (p.n_views, model.n_fov, m_rays),
                  "hbm_alg_frac": p_bytes / (p_ms * 1e-3) / 8e12,
                  "traffic": p_traffic,
                  "hbm_counter_frac": (None if p_traffic is None
                                       else p_traffic / (p_ms * 1e-3) / 8e12),
                  "valu_busy_counter": _fig(figs, p_kernels[1:], "valu_busy")},
            "PT": {"kernels": pt_kernels, "ms": pt_ms, "bound": "alu",
                   "hbm_alg_bytes": pt_bytes,
                   "hbm_alg_note": "the residual read once, v written once",
                   "hbm_alg_frac": pt_bytes / (pt_ms * 1e-3) / 8e12,
                   "traffic": pt_traffic,
                   "hbm_counter_frac": (None if pt_traffic is None
                                        else pt_traffic / (pt_ms * 1e-3) / 8e12),
                   "valu_busy_counter": _fig(figs, pt_kernels[1:], "valu_busy")},
            "VJP": {"ms": v_ms, "bound": "mfma", "flop": vjp_flop,
                    "achieved_tflops": vjp_flop / (v_ms * 1e-3) / 1e12,
                    "frac": vjp_flop / (v_ms * 1e-3) / PEAK[dtype],
                    "traffic": _fig(figs, ["k_vjp_w", "k_dw_gemm2", "k_dw_reduce2"],
                                    "traffic_bytes")},
        }
    out = {
        "metric": ("grad steps/s at 501^3 cone-beam 20 views" if a.config == "c4"
                   else "grad steps/s at " + p.name)
                  + (" (%d ordered subsets)" % a.subsets if a.subsets > 1 else "")
                  + (" (FLS loss)" if a.loss == "fls" else ""),
        "value": 1e3 / ms_step,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (seeded %s phantom, closed-form chord data, %s)"
                % ("ellipsoid" if p.dim == 3 else "ellipse",
                   "Poisson %.0e" % p.photons if p.photons else "noiseless"),
        "config": {"workload": p.name, "grid": "%d^%d" % (p.N, p.dim),
                   "views": p.n_views, "detector": "%dx%d" % (p.n_v, p.n_u),
                   "n_fov": model.n_fov, "k": k, "params": model.n_params,
                   "v_mode": a.v_mode, "subsets": a.subsets, "loss": a.loss,
                   "parallelism": "single GPU"},
        "stages_ms_per_step": {k_: v / a.steps for k_, v in stages.items()},
        "device_mem_gb": (free0 - free1) / 1e9,
        # the library allocates only when handles are created, so the
        # footprint after the timed steps is the peak of the whole run
        "peak_device_mem_gb": (free0 - min(free1, free2)) / 1e9,
        "loss_last": loss,
        "roofline": roofline,
    }
    if stage_roofs is not None:
        out["roofline_stages"] = stage_roofs
    if alt is not None:
        out["v_at_I"] = alt
    if not a.no_cpu:
        log("timing the FP64 oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(p, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
