"""Writes c2_fit_oracle.json: the FP64 oracle's fit of the 2D 512^2 SIREN
workload (parallel beam, 90 views, 725 bins, Poisson data at 1e5 photons;
SIREN 2 -> 5 x 256 -> 1, omega0 30; |I| = n/16 per step; Adam lr 1e-4;
Algorithm 1 + Adam for 2000 steps), recording the image MSE against the
rasterised phantom (over the FOV) every 20 steps.

Calls only the oracle and the seeded input generators; nothing here comes
from the GPU path.  Most of a step is the image evaluation E (the SIREN over
all 206k FOV pixels); with --threads T the oracle's own forward pass runs on T
chunks of the pixel list at once (rows are independent, so only the BLAS
blocking changes).  On seven threads of an 8-core host a step takes about
3.5 s and the fit about two hours; single-threaded about 15-20 s a step.  The
committed record was written by

    OPENBLAS_NUM_THREADS=1 python tests/golden/make_c2_fit.py --threads 7

(defaults: --steps 2000 --every 20, written next to this script).
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import inr as oinr  # noqa: E402
from oracle import sampler as osampler  # noqa: E402
from oracle import step as ostep  # noqa: E402
from paper_2604_09884_amd import configs, synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


class ChunkedProblem(ostep.Problem):
    """The oracle's Problem with E evaluated on chunks of the FOV pixel list
    in a thread pool; every chunk is the oracle's inr.forward."""

    def __init__(self, cfg, threads):
        super().__init__(cfg)
        self.pool = cf.ThreadPoolExecutor(threads)
        self.chunks = np.array_split(np.arange(self.n), 8 * threads)

    def E(self, theta, B):
        parts = self.pool.map(lambda c: oinr.forward(theta, B, self.X[c], self.arch), self.chunks)
        u = np.zeros(self.N ** self.dim)
        u[self.fov] = np.concatenate(list(parts))
        return u


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=20)
    ap.add_argument("--threads", type=int, default=1)
    ap.add_argument("--out", default=os.path.join(HERE, "c2_fit_oracle.json"))
    a = ap.parse_args()
    p = configs.C2
    t0 = time.time()
    prob = ChunkedProblem(p, a.threads) if a.threads > 1 else ostep.Problem(p)
    theta, B = synth.init_inr(p.arch, p.seed_init)
    y = synth.sinogram(p).astype(np.float32).astype(np.float64).ravel()
    truth = synth.raster(synth.phantom(p), 2, p.N)
    k = p.k(prob.n)
    print("C2 oracle: n %d, k %d, rays %d, set-up %.1f s" % (prob.n, k, y.size, time.time() - t0),
          flush=True)
    th, m, v = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    record = {"config": p.name, "steps": a.steps, "k": int(k), "n": int(prob.n),
              "lr": p.lr, "mse": {}, "loss": {}}
    record["mse"]["0"] = ostep.mse(prob.E(th, B), truth, prob.fov)
    for t in range(a.steps):
        idx = osampler.sample_indices(prob.fov, k, p.seed_sampler, t)
        th, m, v, L, _ = ostep.grad_step(prob, th, B, m, v, t + 1, y, idx, p.lr)
        if (t + 1) % a.every == 0 or t + 1 == a.steps:
            record["mse"][str(t + 1)] = ostep.mse(prob.E(th, B), truth, prob.fov)
            record["loss"][str(t)] = L
            print("step %d: loss %.6g, MSE %.6g (%.0f s)" % (t + 1, L, record["mse"][str(t + 1)],
                                                             time.time() - t0), flush=True)
            with open(a.out, "w") as f:
                json.dump(record, f, indent=1)


if __name__ == "__main__":
    main()
