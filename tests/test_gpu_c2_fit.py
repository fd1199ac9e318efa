"""The 2D 512^2 SIREN workload fitted for its full 2000 steps (Algorithm 1 +
Adam, |I| = n/16, parallel beam, 90 views, Poisson data) on the GPU with
the MLP in FP32 and in BF16, against the FP64 oracle's fit of the same
workload from the same seeded inputs.

The fit of this workload is chaotic: an FP32 run follows the FP64 one to
about 1e-4 in MSE until the first of the transient loss excursions that
SIREN + Adam at this learning rate goes through every few hundred steps,
and a 1e-6 relative change of the initial parameters moves such an
excursion by a hundred steps.  Whether one run is inside an excursion at
one given step is therefore chance.  What is compared is the fit's outcome:
the median of the image MSE over the checkpoints of the last 400 steps
(every 20 steps, 21 values), which agrees within 2%.  The MSE at the last
step itself is reported alongside.

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
MIN_TAIL_POINTS = 21


def _oracle_record():
    if not os.path.exists(GOLDEN):
        pytest.skip("no oracle fit record at %s" % GOLDEN)
    rec = json.load(open(GOLDEN))
    steps = rec["steps"]
    recorded = sorted(int(s) for s in rec["mse"])
    if recorded[-1] != steps:
        pytest.skip("the oracle's fit record stops at step %d of %d" % (recorded[-1], steps))
    tail = [s for s in recorded if s >= steps - TAIL]
    if len(tail) < MIN_TAIL_POINTS:
        pytest.skip("the oracle's fit record has %d checkpoints in its last %d steps"
                    % (len(tail), TAIL))
    return rec, tail


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_c2_fit_tail_median_mse_within_2_percent(dtype):
    from paper_2604_09884_amd import ops
    rec, tail = _oracle_record()
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
    checkpoints = set(tail) | {s for s in range(500, rec["steps"], 500)}
    mine = {}
    for t in range(rec["steps"]):
        st.step(t)
        if t + 1 in checkpoints:
            u = host(ops.inr_eval_grid(m, st.theta, st.B))
            mine[t + 1] = ostep.mse(u, truth, fov)
            if (t + 1) % 100 == 0:
                say("C2 %s step %d: MSE %.6g (oracle %.6g)"
                    % (dtype, t + 1, mine[t + 1], rec["mse"].get(str(t + 1), float("nan"))))
    torch.cuda.synchronize()
    st.close()
    med = float(np.median([mine[s] for s in tail]))
    ref = float(np.median([rec["mse"][str(s)] for s in tail]))
    d = abs(med - ref) / ref
    last = rec["steps"]
    d_last = abs(mine[last] - rec["mse"][str(last)]) / rec["mse"][str(last)]
    say("C2 %s median MSE over steps %d-%d: %.6g, oracle %.6g, relative difference %.4f; "
        "at step %d: %.6g, oracle %.6g, relative difference %.4f"
        % (dtype, tail[0], tail[-1], med, ref, d, last, mine[last], rec["mse"][str(last)],
           d_last))
    report("par2d-512-siren (C2) %d-step fit" % last, dtype,
           "median MSE over the last %d steps" % TAIL, d, 0.02)
    report("par2d-512-siren (C2) %d-step fit" % last, dtype, "MSE at the last step", d_last)
    assert d <= 0.02
