"""Stationary equation with ECS and its FFT-preconditioned conjugate-gradient
solve (Sec. III).  Test infrastructure only.

Sec. III: [K_s + U(z(x), t_max) - E] psi_E = f becomes A psi = f with
A = F^-1 K F + C + U - E I (Eq. linsys); A is complex symmetric, and the paper
solves it by preconditioned conjugate gradients with
P^-1 = F^-1 (K - E I)^-1 F (Eq. PreconFFT), [(K - E)^-1]_nn = 1/(k_n^2/2 - E).

Readings:
* "PCG" for a complex-symmetric A is read as COCG: the conjugate-gradient
  recurrences with the unconjugated bilinear form u^T v, which needs a
  symmetric P^-1 (true here because k^2 is even in k).  Start x0 = 0; stop when
  the Hermitian 2-norm ||r|| / ||f|| <= rtol, then recompute the true residual
  f - A x and restart from it while it still exceeds rtol.
* 2D: K = (k_x^2 + k_y^2)/2 and C = C_x (x) I + I (x) C_y as in the TDSE;
  U = V0(z_x, z_y) + f x with the field value f (zero once the pulse is over).
* 3D (Sec. III: the FFT preconditioner generalises to the many-dimensional
  case): K = (k_x^2 + k_y^2 + k_z^2)/2, C = C_x + C_y + C_z, arrays
  [nz][ny][nx]; P^-1 = F^-1 (K - E)^-1 F with the full 3D transform.
* The preconditioner's divisor k^2/2 - E is used as printed.  The optional
  shift eta (divisor k^2/2 - E - i eta) is not from the paper; eta = 0 is the
  printed form.  The shifted symbol is still even in k, so P^-1 stays
  complex symmetric and COCG still applies.
"""
import numpy as np

from . import grid


class Operator:
    """A = F^-1 K F + C + U - E (Sec. III, Eq. linsys) for a 1D or 2D problem
    built from ``oracle.tdse`` axes, and the FFT preconditioner."""

    def __init__(self, axes, V, E, eta=0.0):
        # axes: (ax,) in 1D or (ax, ay) in 2D; V: static potential on the grid;
        # eta: shift of the preconditioner's divisor (0: as printed).
        self.axes = axes
        self.V = np.asarray(V, dtype=complex)
        self.E = complex(E)
        self.eta = float(eta)
        if len(axes) == 1:
            self.K = axes[0].k ** 2 / 2
        elif len(axes) == 2:
            ax, ay = axes
            self.K = (ax.k[None, :] ** 2 + ay.k[:, None] ** 2) / 2
        else:
            ax, ay, az = axes
            self.K = (ax.k[None, None, :] ** 2 + ay.k[None, :, None] ** 2 + az.k[:, None, None] ** 2) / 2

    def _F(self, v):
        # axis a of the grid is array axis ndim - 1 - a (x fastest)
        nd = len(self.axes)
        for a, ax in enumerate(self.axes):
            v = grid.forward(v, ax.L, axis=nd - 1 - a)
        return v

    def _Finv(self, v):
        nd = len(self.axes)
        for a, ax in reversed(list(enumerate(self.axes))):
            v = grid.inverse(v, ax.L, axis=nd - 1 - a)
        return v

    def _C(self, v):
        # C = sum over axes of C_a acting along axis a
        nd = len(self.axes)
        out = np.zeros_like(v, dtype=complex)
        for a, ax in enumerate(self.axes):
            w = np.moveaxis(v, nd - 1 - a, 0)
            shape = w.shape
            cw = (ax.C @ w.reshape(shape[0], -1)).reshape(shape)
            out = out + np.moveaxis(cw, 0, nd - 1 - a)
        return out

    def matvec(self, v):
        """A v = F^-1 K F v + C v + (U - E) v (Sec. III, Eq. linsys)."""
        v = np.asarray(v, dtype=complex)
        return self._Finv(self.K * self._F(v)) + self._C(v) + (self.V - self.E) * v

    def precond(self, r):
        """P^-1 r = F^-1 (K - E)^-1 F r (Sec. III, Eq. PreconFFT); with a shift,
        F^-1 (K - E - i eta)^-1 F r."""
        if self.eta == 0.0:
            return self._Finv(self._F(r) / (self.K - self.E))
        return self._Finv(self._F(r) / (self.K - self.E - 1j * self.eta))

    def dense(self):
        """A as a dense matrix, column by column (tiny grids only)."""
        shape = self.V.shape
        n = self.V.size
        A = np.empty((n, n), dtype=complex)
        for j in range(n):
            e = np.zeros(n, dtype=complex)
            e[j] = 1.0
            A[:, j] = self.matvec(e.reshape(shape)).ravel()
        return A


def dense_solve(op, f):
    """Gaussian elimination on the dense A (Sec. III: the N^3 route)."""
    A = op.dense()
    return np.linalg.solve(A, np.asarray(f, dtype=complex).ravel()).reshape(op.V.shape)


def cocg(op, f, rtol=1e-8, maxit=10000, precond=True):
    """Preconditioned conjugate gradients for complex-symmetric A (COCG
    reading of Sec. III).  Returns (x, iterations, true relative residual)."""
    dot = lambda u, v: np.sum(u * v)                     # unconjugated u^T v
    nrm = lambda u: np.sqrt(np.sum(np.abs(u) ** 2))      # Hermitian 2-norm
    Pinv = op.precond if precond else (lambda r: r)
    f = np.asarray(f, dtype=complex)
    fn = nrm(f)
    x = np.zeros_like(f)
    r = f.copy()
    it = 0
    while True:
        z = Pinv(r)
        p = z.copy()
        rho = dot(r, z)
        while it < maxit:
            w = op.matvec(p)
            alpha = rho / dot(p, w)
            x = x + alpha * p
            r = r - alpha * w
            it += 1
            if nrm(r) / fn <= rtol:
                break
            z = Pinv(r)
            rho_new = dot(r, z)
            p = z + (rho_new / rho) * p
            rho = rho_new
        r = f - op.matvec(x)
        true = nrm(r) / fn
        if true <= rtol or it >= maxit:
            return x, it, true
