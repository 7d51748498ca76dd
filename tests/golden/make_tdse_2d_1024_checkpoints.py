"""Write tdse_2d_1024_checkpoints.npz: the FP64 oracle's state of the 2D
workload (1024 x 1024, h = 0.2, soft-core a2 = 0.64, 4-cycle pulse along x,
SECS from 80% of the half-width with end angle 0.5, packet seed 1, dt = 0.05)
after 100, 500, 1000 and 2000 steps, sampled at 8192 seeded grid points, with
the squared norm of the whole state at each checkpoint.

Calls only the oracle and the seeded input generators.  Takes about ten
minutes on one core:  python tests/golden/make_tdse_2d_1024_checkpoints.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import tdse as ot  # noqa: E402
from paper_1505_06707_amd import workloads as wl  # noqa: E402

CHECKPOINTS = (100, 500, 1000, 2000)
NSAMPLES = 8192
OUT = os.path.join(HERE, "tdse_2d_1024_checkpoints.npz")


def sample_index(n, count=NSAMPLES, seed=77):
    """Flat indices of the sampled grid points (seeded, without repeats)."""
    return np.sort(np.random.default_rng(seed).choice(n * n, size=count, replace=False))


def main():
    c = wl.TDSE_2D
    ax = ot.Axis(c.n, c.L, R0=c.R0, theta=c.theta)
    prob = ot.Problem2D(ax, ax, Zc=c.charge, a2=c.a2)
    psi = wl.gaussian_2d(ax.x, ax.x, **wl.packet_params(1))
    f = c.pulse.at_midpoints(0.0, c.dt, max(CHECKPOINTS))
    idx = sample_index(c.n)
    samples, norms = [], []
    t0 = time.time()
    done = 0
    for cp in CHECKPOINTS:
        psi = prob.propagate(psi, c.dt, f[done:cp])
        done = cp
        samples.append(psi.ravel()[idx])
        norms.append(float(np.sum(np.abs(psi) ** 2)))
        print(f"step {cp}: norm^2 {norms[-1]:.12f} ({time.time() - t0:.0f} s)", flush=True)
    np.savez(OUT, steps=np.array(CHECKPOINTS), index=idx, samples=np.array(samples), norm2=np.array(norms),
             packet_seed=1)


if __name__ == "__main__":
    main()
