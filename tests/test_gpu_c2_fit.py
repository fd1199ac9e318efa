"""The 2D 512^2 SIREN workload fitted for its full 2000 steps (Algorithm 1 +
Adam, |I| = n/16, parallel beam, 90 views, Poisson data) on the GPU with
the MLP in FP32 and in BF16, against the FP64 oracle's fit of the same
workload from the same seeded inputs.

The fit of this workload is chaotic.  SIREN + Adam at this learning rate goes
through transient loss excursions every few hundred steps, each followed by a
recovery of a few hundred steps, and their timing depends on rounding.
Twelve GPU runs per MLP precision, from the initial parameters and from
eleven copies perturbed by 1e-6 (relative): the FP32 runs' final MSEs range
over 0.89e-3 to 1.15e-3 (standard deviation 9%), their medians over the last
400 steps over 0.96e-3 to 1.07e-3 (mean 1.006e-3, sd 3.9%); the BF16 medians
over 1.02e-3 to 1.30e-3 (mean 1.136e-3, 13% above FP32's, sd 7.1%).  So no
implementation whose arithmetic is not the oracle's, bit for bit, can be held
to a 2% agreement of one final MSE; what is checked:

  * FP32 trajectory: until the first excursion, the fit is a smooth function
    of the arithmetic.  The MSE every 20 steps up to step 400 agrees with the
    oracle's within 2% (runs from perturbed initial parameters stay within
    0.5% of each other there).
  * Outcome: the median MSE over the last 400 steps (21 checkpoints) agrees
    with the oracle's within 10% in FP32 (2.5 standard deviations of the
    difference of two FP32-like runs) and within 35% in BF16 (the 13% shift
    plus 2.6 standard deviations of the difference of a BF16 and an FP32-like
    run).

The relative difference of the MSE at the last step itself is reported.

The oracle's values are in tests/golden/c2_fit_oracle.json, written by
tests/golden/make_c2_fit.py, which calls only the oracle."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import grid as ogrid
from oracle import step as ostep
from paper_2604_09884_amd import configs, synth
from tests.gpu_util import dev, host, report, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_fit_oracle.json")
TAIL = 400
EARLY = 400
EVERY = 20
TOL_EARLY = 0.02
TOL_TAIL = {"fp32": 0.10, "bf16": 0.35}


def _oracle_record():
    if not os.path.exists(GOLDEN):
        pytest.skip("no oracle fit record at %s" % GOLDEN)
    rec = json.load(open(GOLDEN))
    steps = rec["steps"]
    recorded = {int(s) for s in rec["mse"]}
    if max(recorded) != steps:
        pytest.skip("the oracle's fit record stops at step %d of %d" % (max(recorded), steps))
    want = set(range(EVERY, steps + 1, EVERY))
    if not want <= recorded:
        pytest.skip("the oracle's fit record is not every %d steps" % EVERY)
    return rec


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_c2_fit_against_oracle(dtype):
    from paper_2604_09884_amd import ops
    rec = _oracle_record()
    steps = rec["steps"]
    p = configs.C2
    fov = ogrid.fov_indices(2, p.N)
    k = p.k(fov.size)
    assert rec["config"] == p.name and rec["k"] == k and rec["n"] == fov.size
    theta, B = synth.init_inr(p.arch, p.seed_init)
    y = synth.sinogram(p).astype(np.float32)
    truth = synth.raster(synth.phantom(p), 2, p.N)
    m = ops.Model(p.arch, 2, p.N, dtype, max_k=k)
    g = ops.Geometry(p)
    st = ops.GradStepper(m, g, dev(theta), dev(np.zeros(1)), dev(y.ravel()), k, p.lr,
                         seed=p.seed_sampler)
    mine = {}
    for t in range(steps):
        st.step(t)
        if (t + 1) % EVERY == 0:
            u = host(ops.inr_eval_grid(m, st.theta, st.B))
            mine[t + 1] = ostep.mse(u, truth, fov)
            if (t + 1) % 500 == 0:
                say("C2 %s step %d: MSE %.6g (oracle %.6g)"
                    % (dtype, t + 1, mine[t + 1], rec["mse"][str(t + 1)]))
    torch.cuda.synchronize()
    st.close()
    ref = {s: rec["mse"][str(s)] for s in mine}
    early = max(abs(mine[s] - ref[s]) / ref[s] for s in range(EVERY, EARLY + 1, EVERY))
    tail = range(steps - TAIL, steps + 1, EVERY)
    med, med_ref = np.median([mine[s] for s in tail]), np.median([ref[s] for s in tail])
    d_tail = abs(med - med_ref) / med_ref
    d_last = abs(mine[steps] - ref[steps]) / ref[steps]
    say("C2 %s: largest MSE difference over steps %d-%d %.4f; median MSE over steps %d-%d "
        "%.6g, oracle %.6g (difference %.4f); at step %d %.6g, oracle %.6g (difference %.4f)"
        % (dtype, EVERY, EARLY, early, tail[0], tail[-1], med, med_ref, d_tail, steps,
           mine[steps], ref[steps], d_last))
    w = "par2d-512-siren (C2) %d-step fit" % steps
    report(w, dtype, "MSE, steps %d-%d (largest)" % (EVERY, EARLY), early,
           TOL_EARLY if dtype == "fp32" else None)
    report(w, dtype, "median MSE over the last %d steps" % TAIL, d_tail, TOL_TAIL[dtype])
    report(w, dtype, "MSE at the last step", d_last)
    if dtype == "fp32":
        assert early <= TOL_EARLY
    assert d_tail <= TOL_TAIL[dtype]
