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
        else:
            ax, ay = axes
            self.K = (ax.k[None, :] ** 2 + ay.k[:, None] ** 2) / 2

    def _F(self, v):
        if len(self.axes) == 1:
            return grid.forward(v, self.axes[0].L)
        ax, ay = self.axes
        return grid.forward(grid.forward(v, ax.L, axis=1), ay.L, axis=0)

    def _Finv(self, v):
        if len(self.axes) == 1:
            return grid.inverse(v, self.axes[0].L)
        ax, ay = self.axes
        return grid.inverse(grid.inverse(v, ay.L, axis=0), ax.L, axis=1)

    def _C(self, v):
        if len(self.axes) == 1:
            return self.axes[0].C @ v
        ax, ay = self.axes
        return (ax.C @ v.T).T + ay.C @ v

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
