"""Seeded synthetic workloads: problem parameters and input generators.

This module holds inputs only (initial packets, pulse samples, sources,
energies, problem sizes).  None of the method's arithmetic lives here; both the
HIP library and the CPU oracle take what it produces as plain arrays.

Workloads (all atomic units):

* ``tdse_1d``  -- 1D TDSE, N = 4096 on [-204.8, 204.8) (h = 0.1), soft-core
  -1/sqrt(x^2 + 2) plus a dipole field E0 sin^2(pi t/T) sin(w t) x with
  E0 = 0.05, w = 0.057, T = 4 cycles; SECS beyond R0 = 150 with end angle 0.5;
  Gaussian of width 1 at rest at the origin; dt = 0.05, 4000 steps.
* ``tdse_2d``  -- 2D TDSE on 1024 x 1024, h = 0.2, soft-core
  -1/sqrt(x^2 + y^2 + 0.64), the same pulse polarised along x, SECS on all
  four edges from 80% of the half-width, end angle 0.5; Gaussian with a seeded
  centre in [-2, 2]^2 and momentum in [-0.5, 0.5]^2; dt = 0.05, 2000 steps.
* ``sse_2d``   -- stationary equation on 512 x 512, h = 0.2, the static part
  of the same potential and contour, smooth seeded source (complex white noise
  filtered by a periodic Gaussian of sigma = 2 cells, unit 2-norm), 128
  energies uniform in [0.05, 2.0], residual 1e-8.
* ``batch_2d`` -- 96 independent 2D runs with square grids drawn by seed from
  {256, 384, 512, 768, 1024}^2 (h = 0.2), E0 ~ U[0.02, 0.1], w ~ U[0.04, 0.08],
  1000 steps each.
* ``learned_2d`` -- stationary equation on 1024 x 1024 at 64 energies in
  [0.05, 2.0] with the ``sse_2d`` source recipe.
* ``tdse_3d``  -- 3D TDSE on 256^3, h = 0.4 (box +-51.2), soft-core
  -1/sqrt(x^2 + y^2 + z^2 + 0.64), the same pulse along x, SECS on all six
  faces from 80% of the half-width, end angle 0.5; Gaussian with a seeded
  centre in [-2, 2]^3 and momentum in [-0.5, 0.5]^3; dt = 0.05.
* ``sse_3d``   -- stationary equation on 128^3, h = 0.4 (box +-25.6), the static
  part of the 3D potential and contour, the ``sse_2d`` source recipe on three
  axes, 16 energies uniform in [0.05, 2.0], residual 1e-8.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Pulse:
    E0: float = 0.05
    omega: float = 0.057
    cycles: float = 4.0

    @property
    def duration(self):
        return self.cycles * 2 * np.pi / self.omega

    def __call__(self, t):
        t = np.asarray(t, dtype=float)
        T = self.duration
        on = (t >= 0) & (t <= T)
        return np.where(on, self.E0 * np.sin(np.pi * t / T) ** 2 * np.sin(self.omega * t), 0.0)

    def at_midpoints(self, t0, dt, nsteps):
        """f(t0 + (n + 1/2) dt), n = 0..nsteps-1: the field of each step."""
        return self(t0 + (np.arange(nsteps) + 0.5) * dt)


@dataclass(frozen=True)
class TDSE1D:
    n: int = 4096
    L: float = 409.6
    R0: float = 150.0
    theta: float = 0.5
    charge: float = 1.0
    a2: float = 2.0
    pulse: Pulse = field(default_factory=Pulse)
    dt: float = 0.05
    nsteps: int = 4000


@dataclass(frozen=True)
class TDSE2D:
    n: int = 1024
    h: float = 0.2
    theta: float = 0.5
    charge: float = 1.0
    a2: float = 0.64
    pulse: Pulse = field(default_factory=Pulse)
    dt: float = 0.05
    nsteps: int = 2000
    R0_frac: float = 0.8

    @property
    def L(self):
        return self.n * self.h

    @property
    def R0(self):
        return self.R0_frac * self.L / 2


@dataclass(frozen=True)
class SSE2D:
    n: int = 512
    h: float = 0.2
    theta: float = 0.5
    charge: float = 1.0
    a2: float = 0.64
    R0_frac: float = 0.8
    n_energies: int = 128
    E_lo: float = 0.05
    E_hi: float = 2.0
    rtol: float = 1e-8
    sigma_cells: float = 2.0

    @property
    def L(self):
        return self.n * self.h

    @property
    def R0(self):
        return self.R0_frac * self.L / 2

    def energies(self):
        return np.linspace(self.E_lo, self.E_hi, self.n_energies)


@dataclass(frozen=True)
class TDSE3D:
    n: int = 256
    h: float = 0.4
    theta: float = 0.5
    charge: float = 1.0
    a2: float = 0.64
    pulse: Pulse = field(default_factory=Pulse)
    dt: float = 0.05
    nsteps: int = 100
    R0_frac: float = 0.8

    @property
    def L(self):
        return self.n * self.h

    @property
    def R0(self):
        return self.R0_frac * self.L / 2


@dataclass(frozen=True)
class SSE3D:
    n: int = 128
    h: float = 0.4
    theta: float = 0.5
    charge: float = 1.0
    a2: float = 0.64
    R0_frac: float = 0.8
    n_energies: int = 16
    E_lo: float = 0.05
    E_hi: float = 2.0
    rtol: float = 1e-8
    sigma_cells: float = 2.0

    @property
    def L(self):
        return self.n * self.h

    @property
    def R0(self):
        return self.R0_frac * self.L / 2

    def energies(self):
        return np.linspace(self.E_lo, self.E_hi, self.n_energies)


TDSE_1D = TDSE1D()
TDSE_3D = TDSE3D()
TDSE_2D = TDSE2D()
SSE_2D = SSE2D()
SSE_3D = SSE3D()
LEARNED_2D = SSE2D(n=1024, n_energies=64)
BATCH_SIZES = (256, 384, 512, 768, 1024)


def gaussian_1d(x, x0=0.0, k0=0.0):
    """pi^{-1/4} exp(-(x - x0)^2/2 + i k0 x) sampled at the given points."""
    x = np.asarray(x, dtype=float)
    return np.pi ** -0.25 * np.exp(-(x - x0) ** 2 / 2 + 1j * k0 * x)


def gaussian_2d(x, y, x0=0.0, y0=0.0, px=0.0, py=0.0):
    """pi^{-1/2} exp(-((x-x0)^2 + (y-y0)^2)/2 + i (px x + py y)) on the [ny][nx]
    grid spanned by the 1D point sets x (fast axis) and y."""
    X = np.asarray(x, dtype=float)[None, :]
    Y = np.asarray(y, dtype=float)[:, None]
    return (np.pi ** -0.5 * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / 2
                                   + 1j * (px * X + py * Y)))


def packet_params(seed):
    """Seeded centre in [-2, 2]^2 and momentum in [-0.5, 0.5]^2."""
    rng = np.random.default_rng(seed)
    x0, y0 = rng.uniform(-2.0, 2.0, size=2)
    px, py = rng.uniform(-0.5, 0.5, size=2)
    return dict(x0=float(x0), y0=float(y0), px=float(px), py=float(py))


def smooth_source(ny, nx, seed, sigma_cells=2.0):
    """Complex white noise (Re, Im ~ N(0,1)) smoothed by a periodic Gaussian
    filter of standard deviation ``sigma_cells`` grid cells, scaled to unit
    2-norm.  Shape [ny][nx] (or [nx] when ny is None)."""
    rng = np.random.default_rng(seed)
    shape = (nx,) if ny is None else (ny, nx)
    w = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    filt = np.exp(-(sigma_cells * kx) ** 2 / 2)
    if ny is not None:
        ky = 2 * np.pi * np.fft.fftfreq(ny)
        filt = filt[None, :] * np.exp(-(sigma_cells * ky) ** 2 / 2)[:, None]
        s = np.fft.ifft2(np.fft.fft2(w) * filt)
    else:
        s = np.fft.ifft(np.fft.fft(w) * filt)
    return s / np.linalg.norm(s)


def batch_runs(seed, nruns=96, sizes=BATCH_SIZES):
    """Seeded list of uneven 2D runs: grid size and pulse per run."""
    rng = np.random.default_rng(seed)
    runs = []
    for r in range(nruns):
        n = int(sizes[rng.integers(len(sizes))])
        E0 = float(rng.uniform(0.02, 0.1))
        omega = float(rng.uniform(0.04, 0.08))
        runs.append(dict(n=n, pulse=Pulse(E0=E0, omega=omega), packet_seed=int(rng.integers(1 << 30))))
    return runs


def packet_params_3d(seed):
    """Seeded centre in [-2, 2]^3 and momentum in [-0.5, 0.5]^3."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-2.0, 2.0, size=3)
    k = rng.uniform(-0.5, 0.5, size=3)
    return dict(x0=float(c[0]), y0=float(c[1]), z0=float(c[2]), px=float(k[0]), py=float(k[1]), pz=float(k[2]))


def gaussian_3d(x, y, z, x0=0.0, y0=0.0, z0=0.0, px=0.0, py=0.0, pz=0.0):
    """pi^{-3/4} exp(-|r - r0|^2/2 + i p.r) on the [nz][ny][nx] grid of the
    1D point sets x (fast), y and z."""
    X = np.asarray(x, dtype=float)[None, None, :]
    Y = np.asarray(y, dtype=float)[None, :, None]
    Z = np.asarray(z, dtype=float)[:, None, None]
    return (np.pi ** -0.75 * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2 + (Z - z0) ** 2) / 2
                                    + 1j * (px * X + py * Y + pz * Z)))


def smooth_source_3d(nz, ny, nx, seed, sigma_cells=2.0):
    """The ``smooth_source`` recipe on a [nz][ny][nx] grid: complex white noise
    smoothed by a periodic Gaussian of ``sigma_cells`` cells along every axis,
    unit 2-norm."""
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(nz, ny, nx)) + 1j * rng.normal(size=(nz, ny, nx))
    filt = 1.0
    for a, n in enumerate((nz, ny, nx)):
        k = 2 * np.pi * np.fft.fftfreq(n)
        shape = [1, 1, 1]
        shape[a] = n
        filt = filt * np.exp(-(sigma_cells * k) ** 2 / 2).reshape(shape)
    s = np.fft.ifftn(np.fft.fftn(w) * filt)
    return s / np.linalg.norm(s)
