"""Writes trajectory_faults10k.txt: the FP64 oracle's pSGLD run on the
faults10k workload (10,000 events, 50 stations, 5,000,000 observations,
6-128x4-1 network), one chain, minibatch 65,536, step 1e-4, beta2 0.99,
eps_p 1e-5, exact whitening (Sec. 3.1, Sec. 3.2 eq:pSGLD), 200 steps with
the batch and noise streams of seed 23 and catalog stream 5; moments over
the states after steps 100..199 (burn-in 100, thin 1, Sec. 3.4).

Stored for 500 events drawn with a fixed seed: the posterior mean (4), the
covariance upper triangle (10, divisor count - 1) and the final state theta
(4) and pSGLD second moment v (4).  Calls only oracle/ and the seeded input
generator.  Run from the repository root:

    python tests/golden/make_trajectory_faults10k.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import likelihood as lk  # noqa: E402
from oracle import sampler  # noqa: E402
from paper_2508_12117_amd import synth  # noqa: E402

SEED, STREAM, STEPS, BURN, THIN, N_EVENTS = 23, 5, 200, 100, 1, 500
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "trajectory_faults10k.txt")


def main():
    cat = synth.make_catalog("faults10k")
    net = synth.net_for(cat)
    prob = lk.load(cat)
    cfg = sampler.SamplerConfig(step=cat.wl.step_size, beta2=cat.wl.beta2, eps_p=cat.wl.eps_p,
                                seed=SEED, burn_in=BURN, thin=THIN)
    ch, _ = sampler.run(prob, net, cfg, cat.wl.batch, STEPS, stream=STREAM, chain_id=0)
    cov = sampler.covariance(ch.mom)
    ev = np.sort(np.random.default_rng(7).choice(cat.M, N_EVENTS, replace=False))
    rows = np.column_stack([ev, ch.mom.mean[ev], cov[ev], ch.theta[ev], ch.v[ev]])
    header = (f"oracle pSGLD run: faults10k, seed {SEED}, stream {STREAM}, chain 0, "
              f"batch {cat.wl.batch}, step {cat.wl.step_size}, {STEPS} steps, burn-in {BURN}, "
              f"thin {THIN}, samples {ch.mom.count}\n"
              "columns: event, mean x y z t, cov xx xy xz xt yy yz yt zz zt tt, "
              "theta x y z t, v x y z t")
    fmt = ["%d"] + ["%.17g"] * (rows.shape[1] - 1)
    np.savetxt(OUT, rows, fmt=fmt, header=header)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
