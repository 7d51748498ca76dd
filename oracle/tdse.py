"""Split-operator SO-FFT + ECS time step (Sec. II), 1D and 2D.  Test
infrastructure only.

Sec. II gives the scheme
    psi(t+tau) = F^-1 e^{-iK tau/2} F . e^{-iU tau/2} . e^{-iC tau}
                 . e^{-iU tau/2} . F^-1 e^{-iK tau/2} F psi(t)
with U evaluated at t + tau/2 and e^{-iC tau} by Crank-Nicolson.  The oracle
applies the five factors one after the other, right to left, with four FFTs per
step and no merging of neighbouring kinetic half-steps.

Readings:
* The printed TDSE lacks the factor i on the left; the propagator
  exp(-i(K+U) tau) fixes i dpsi/dt = (K + U) psi.
* Both potential half-steps use U(t + tau/2).
* Potential: U(x, t) = V0(z(x)) + f(t) x.  The static part is evaluated on
  the complex contour, as the scaled equation prescribes (U(z(x), t)); the
  dipole term of an external field is kept at the real coordinate x (on z it
  grows without bound in the scaled region).  V0 is a soft-core Coulomb
  potential -Zc/sqrt(z^2 + a2) in 1D and -Zc/sqrt(z_x^2 + z_y^2 + a2) in 2D,
  principal square-root branch.
* 2D (the paper is 1D): the scaling is separable, q = q(x) q(y),
  K_s = K_s^x + K_s^y, so C = C_x (x) I + I (x) C_y, and since the two terms
  commute e^{-iC tau} is taken as CN(C_x) CN(C_y), one CN sweep along each
  axis.  Arrays are [ny][nx] with x the fast (last) axis; the field is
  polarised along x.
* 3D (the paper's conclusion names the many-dimensional case as the next
  step; Sec. III says the FFT preconditioner generalises to it): the same
  separable reading, K = (k_x^2 + k_y^2 + k_z^2)/2, C = C_x + C_y + C_z, and
  e^{-iC tau} taken as CN(C_x) CN(C_y) CN(C_z).  Arrays are [nz][ny][nx].
* Grid values are the values psi~(x_j) = sqrt(q) psi(z(x_j)) of the scaled
  function (Sec. II, Eq. psi_zx); the scheme is linear, so the DVR factor
  sqrt(h) of the coefficients is immaterial.
"""
import numpy as np

from . import contour, ecs, grid


class Axis:
    """One Cartesian axis: grid, momenta, contour tables and the CN factor."""

    def __init__(self, n, L, kind=contour.SECS, R0=None, theta=0.5):
        self.n, self.L = int(n), float(L)
        self.h = self.L / self.n
        self.kind, self.theta = kind, float(theta)
        self.rmax = self.L / 2
        self.R0 = self.rmax if R0 is None else float(R0)
        self.x = grid.nodes(self.n, self.L)
        self.xm = grid.midpoints(self.n, self.L)
        self.k = grid.momenta(self.n, self.L)
        args = (kind, self.R0, self.rmax, self.theta, self.h)
        self.q = contour.q_of_x(self.x, *args)
        self.qm = contour.q_of_x(self.xm, *args)
        self.z = contour.z_of_x(self.x, *args)
        self.C = ecs.remainder_matrix(self.q, self.qm, self.h)
        self._cn = {}

    def cn(self, tau):
        if tau not in self._cn:
            self._cn[tau] = ecs.CrankNicolson(self.C, tau)
        return self._cn[tau]


def softcore(Zc, a2, *zs):
    """V0 = -Zc / sqrt(sum z^2 + a2) at complex coordinates (principal branch)."""
    if Zc == 0:
        return np.zeros(np.broadcast(*zs).shape, dtype=complex)
    s = a2 + sum(z * z for z in zs)
    return -Zc / np.sqrt(s.astype(complex))


class Problem1D:
    """U(x, t) = V0 + f(t) W: by default the soft-core V0 at z(x) and W = x;
    ``V0`` (complex, at z) and ``W`` (real) on the grid replace them."""

    def __init__(self, axis, Zc=1.0, a2=2.0, V0=None, W=None):
        self.ax = axis
        self.V0 = softcore(Zc, a2, axis.z) if V0 is None else np.asarray(V0, dtype=complex)
        self.W = axis.x if W is None else np.asarray(W, dtype=float)

    def potential(self, f):
        return self.V0 + f * self.W

    def step(self, psi, tau, f_mid):
        ax = self.ax
        kin = np.exp(-1j * ax.k**2 / 2 * tau / 2)     # e^{-iK tau/2}
        pot = np.exp(-1j * self.potential(f_mid) * tau / 2)
        psi = grid.inverse(kin * grid.forward(psi, ax.L), ax.L)
        psi = pot * psi
        psi = ax.cn(tau).apply(psi)
        psi = pot * psi
        psi = grid.inverse(kin * grid.forward(psi, ax.L), ax.L)
        return psi

    def propagate(self, psi, tau, f_mid):
        psi = np.asarray(psi, dtype=complex)
        for f in f_mid:
            psi = self.step(psi, tau, f)
        return psi


class Problem2D:
    """U = V0 + f(t) W on the [ny][nx] grid: by default the soft-core V0 at
    (z_x, z_y) and W = x; ``V0`` (complex) and ``W`` (real) replace them."""

    def __init__(self, axis_x, axis_y, Zc=1.0, a2=0.64, V0=None, W=None):
        self.ax, self.ay = axis_x, axis_y
        self.V0 = (softcore(Zc, a2, axis_x.z[None, :], axis_y.z[:, None]) if V0 is None
                   else np.asarray(V0, dtype=complex))
        self.W = np.broadcast_to(axis_x.x[None, :], self.V0.shape) if W is None else np.asarray(W, dtype=float)
        self.K = (axis_x.k[None, :] ** 2 + axis_y.k[:, None] ** 2) / 2

    def potential(self, f):
        return self.V0 + f * self.W

    def _kinetic(self, psi, phase):
        ax, ay = self.ax, self.ay
        spec = grid.forward(grid.forward(psi, ax.L, axis=1), ay.L, axis=0)
        return grid.inverse(grid.inverse(phase * spec, ay.L, axis=0), ax.L, axis=1)

    def step(self, psi, tau, f_mid):
        kin = np.exp(-1j * self.K * tau / 2)
        pot = np.exp(-1j * self.potential(f_mid) * tau / 2)
        psi = self._kinetic(psi, kin)
        psi = pot * psi
        psi = self.ax.cn(tau).apply(psi, axis=1)
        psi = self.ay.cn(tau).apply(psi, axis=0)
        psi = pot * psi
        psi = self._kinetic(psi, kin)
        return psi

    def propagate(self, psi, tau, f_mid):
        psi = np.asarray(psi, dtype=complex)
        for f in f_mid:
            psi = self.step(psi, tau, f)
        return psi



class Problem3D:
    """U = V0 + f(t) W on the [nz][ny][nx] grid: by default the soft-core V0
    at (z_x, z_y, z_z) and W = x (polarisation along x); ``V0`` (complex) and
    ``W`` (real) replace them."""

    def __init__(self, axis_x, axis_y, axis_z, Zc=1.0, a2=0.64, V0=None, W=None):
        self.ax, self.ay, self.az = axis_x, axis_y, axis_z
        shape = (axis_z.n, axis_y.n, axis_x.n)
        self.V0 = (softcore(Zc, a2, axis_x.z[None, None, :], axis_y.z[None, :, None], axis_z.z[:, None, None])
                   if V0 is None else np.asarray(V0, dtype=complex))
        self.V0 = np.broadcast_to(self.V0, shape)
        self.W = np.broadcast_to(axis_x.x[None, None, :], shape) if W is None else np.asarray(W, dtype=float)
        self.K = (axis_x.k[None, None, :] ** 2 + axis_y.k[None, :, None] ** 2 + axis_z.k[:, None, None] ** 2) / 2

    def potential(self, f):
        return self.V0 + f * self.W

    def _kinetic(self, psi, phase):
        ax, ay, az = self.ax, self.ay, self.az
        spec = grid.forward(grid.forward(grid.forward(psi, ax.L, axis=2), ay.L, axis=1), az.L, axis=0)
        spec = phase * spec
        return grid.inverse(grid.inverse(grid.inverse(spec, az.L, axis=0), ay.L, axis=1), ax.L, axis=2)

    def step(self, psi, tau, f_mid):
        kin = np.exp(-1j * self.K * tau / 2)
        pot = np.exp(-1j * self.potential(f_mid) * tau / 2)
        psi = self._kinetic(psi, kin)
        psi = pot * psi
        psi = self.ax.cn(tau).apply(psi, axis=2)
        psi = self.ay.cn(tau).apply(psi, axis=1)
        psi = self.az.cn(tau).apply(psi, axis=0)
        psi = pot * psi
        psi = self._kinetic(psi, kin)
        return psi

    def propagate(self, psi, tau, f_mid):
        psi = np.asarray(psi, dtype=complex)
        for f in f_mid:
            psi = self.step(psi, tau, f)
        return psi
