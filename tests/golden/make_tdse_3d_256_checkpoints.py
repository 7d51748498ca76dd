"""Write tdse_3d_256_checkpoints.npz: the FP64 oracle's state of the 3D
workload (256^3, h = 0.4, soft-core a2 = 0.64, 4-cycle pulse along x, SECS
from 80% of the half-width with end angle 0.5, packet seed 3, dt = 0.05)
after 25, 50 and 100 steps, sampled at 8192 seeded grid points, with the
squared norm of the whole state at each checkpoint.

Calls only the oracle and the seeded input generators (scipy.fft on every
core; about 12 minutes on 8 cores):
    python tests/golden/make_tdse_3d_256_checkpoints.py
"""
import os
import sys
import time

import numpy as np
import scipy.fft

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import tdse as ot  # noqa: E402
from paper_1505_06707_amd import workloads as wl  # noqa: E402

CHECKPOINTS = (25, 50, 100)
NSAMPLES = 8192
SEED = 3
OUT = os.path.join(HERE, "tdse_3d_256_checkpoints.npz")


def main():
    c = wl.TDSE_3D
    ax = ot.Axis(c.n, c.L, R0=c.R0, theta=c.theta)
    prob = ot.Problem3D(ax, ax, ax, Zc=c.charge, a2=c.a2)
    psi = wl.gaussian_3d(ax.x, ax.x, ax.x, **wl.packet_params_3d(SEED))
    f = c.pulse.at_midpoints(0.0, c.dt, max(CHECKPOINTS))
    idx = np.sort(np.random.default_rng(78).choice(c.n ** 3, size=NSAMPLES, replace=False))
    samples, norms = [], []
    t0 = time.time()
    done = 0
    with scipy.fft.set_workers(os.cpu_count()):
        for cp in CHECKPOINTS:
            psi = prob.propagate(psi, c.dt, f[done:cp])
            done = cp
            samples.append(psi.ravel()[idx])
            norms.append(float(np.sum(np.abs(psi) ** 2)))
            print(f"step {cp}: norm^2 {norms[-1]:.12f} ({time.time() - t0:.0f} s)", flush=True)
    np.savez(OUT, steps=np.array(CHECKPOINTS), index=idx, samples=np.array(samples), norm2=np.array(norms),
             packet_seed=SEED)


if __name__ == "__main__":
    main()
