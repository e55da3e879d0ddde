"""Plain reference of the charge-initialisation policy (paper: Ionic Charge
Initialization section, Algorithm 1) and of the initial walker placement
(Electron Sampler section).

TEST INFRASTRUCTURE ONLY: imported by the tests; the product path never
imports it.  Written from the algorithm's steps in the paper's order.
"""
from __future__ import annotations

import numpy as np

from . import oracle as _o


def electron_counts(partial_charge, atomic_number, t):
    """Algorithm 1: `charge` is the partial-charge vector, `electron` starts
    as the atomic numbers, t is the ion's charge; loop until t = 0."""
    charge = [float(c) for c in partial_charge]
    electron = [int(z) for z in atomic_number]
    while t != 0:
        if t < 0:
            index = min(range(len(charge)), key=lambda m: (charge[m], m))     # argmin, first index on ties
            electron[index] += 1
            t += 1
            charge[index] += 1
        else:
            index = max(range(len(charge)), key=lambda m: (charge[m], -m))    # argmax, first index on ties
            electron[index] -= 1
            t -= 1
            charge[index] -= 1
    return electron


def init_walkers(nuc_xyz, site, scale, seed, stream_id, walkers):
    """[B][N][3]: electron i at nucleus site[i] plus scale z, z the sampler's
    normal deviates of walker w at counter step 0xFFFFFFFF."""
    nuc_xyz = np.asarray(nuc_xyz, dtype=np.float64).reshape(-1, 3)
    centres = nuc_xyz[np.asarray(site, dtype=np.int64)].reshape(-1)
    n3 = centres.size
    out = np.empty((walkers, n3))
    for w in range(walkers):
        z, _ = _o.draw_one(seed, stream_id, w, n3, 0xFFFFFFFF)
        out[w] = centres + scale * z
    return out.reshape(walkers, -1, 3)
