"""Writes tests/golden/equilibrated_walkers.npz: walker positions that sample
|psi|^2 of the seeded random-init networks (Electron Sampler section: the
Metropolis-Hastings chain run from the electrons' initial placement about
the nuclei), produced by the FP64 oracle's chain only.

    python tests/golden/make_equilibrated_walkers.py

Each system starts from its seeded initial walkers (inputs.init_walkers,
walker seed 10287) with the seeded parameters (theta seed 2401, rounded to
FP32 as the FP32 and mixed modes see them) and runs STEPS moves of
sigma = 0.2 bohr with Philox seed CHAIN_SEED, stream 0.  Seeded inputs
stand in for the paper's sampled electrons (it publishes no walker data).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                        # noqa: E402
from paper_2401_10287_amd import inputs as I          # noqa: E402

CHAIN_SEED = 2024
SIGMA = 0.2
# (system, walkers, steps); the serving mix's atoms and ions (Z 2..10,
# charge -1..+2) as "Z<z>q<charge>" with 6 walkers each
PLAN = (("LiH", I.lih, 4096, 300), ("LiF", I.lif, 512, 300), ("H20", I.h_chain, 128, 300)) + tuple(
    (f"Z{z}q{q:+d}", (lambda z=z, q=q: I.atom_ion(z, q, walkers=6)), 6, 200) for z, q in I.serving_job_types())


def main():
    out = {}
    for name, make, walkers, steps in PLAN:
        s = make()
        th = I.init_params(s).astype(np.float32).astype(np.float64)
        o = O.Oracle(s)
        x = I.init_walkers(s, walkers)
        la = o.log_psi(th, x)["log_abs"]
        t = time.time()
        acc = np.zeros(walkers)
        for k in range(0, steps, 50):
            x, la, a = o.metropolis(th, x, la, 50, SIGMA, seed=CHAIN_SEED, step0=k)
            acc += a
            if walkers > 6:
                print(f"{name}: {k + 50} of {steps} steps, {time.time() - t:.0f} s", flush=True)
        out[name] = x
        out[name + "_steps"] = np.array(steps)
        out[name + "_acceptance"] = np.array(acc.mean() / steps)
    out["chain_seed"] = np.array(CHAIN_SEED)
    out["sigma"] = np.array(SIGMA)
    np.savez_compressed(os.path.join(HERE, "equilibrated_walkers.npz"), **out)


if __name__ == "__main__":
    main()
