"""The banded ECS eigen-preconditioner of Sec. III (Eqs. Prec_eigen_eq, K_l,
PreconFFT_ECS), in FP64.  Test infrastructure only.

Per axis the spectrum (FFT index order, k_0 = 0 first) is cut into bands of
consecutive momenta.  On a band the matrix
    [K_l]_{nm} = 1/2 k_n k_m Q_{nm},   Q_{nm} = int phi_n^* q(x)^-2 phi_m dx,
is the Fourier-basis block of K_a = -1/2 d/dx q^-2 d/dx.  Its eigenvectors chi,
normalised by chi^T chi = 1, are the rows of the block of X, and
    P^-1 = F^-1 X^T (Lambda - E)^-1 X F.
In 2D the kinetic operator is K_x + K_y, so X = X_x (x) X_y and the divisor is
lambda_x + lambda_y - E; in 3D (Sec. III's many-dimensional case, read the same
way) X = X_x (x) X_y (x) X_z and the divisor lambda_x + lambda_y + lambda_z - E.

Readings:
* Q_{nm} depends on k_m - k_n only (Toeplitz).  It is evaluated by the grid
  quadrature of the DVR basis: Q(d) = (1/N) sum_j q(x_j)^-2 exp(i 2 pi d x_j / L).
* Bands: the paper's split.  {k_0} and {k_N/2} alone; the positive momenta,
  from k_1 outward, in bands of N_BW = 10 with the remainder joined to the band
  next to k_N/2 (width 10..19); the negative momenta mirror the positive ones.
  Axes with fewer than N_BW positive momenta use one band per sign.
* Eigen-decomposition of each complex-symmetric block by a general eigensolver,
  each eigenvector divided by sqrt(chi^T chi) (principal branch).
"""
import numpy as np

N_BW = 10


def bands(n, nbw=N_BW):
    """Index lists of the bands of an axis with n nodes (FFT order)."""
    half = n // 2
    pos = list(range(1, half))
    nfull = len(pos) // nbw
    if nfull == 0:
        groups = [pos] if pos else []
    else:
        groups = [pos[i * nbw:(i + 1) * nbw] for i in range(nfull - 1)] + [pos[(nfull - 1) * nbw:]]
    out = [[0], [half]]
    for g in groups:
        out.append(list(g))
        out.append(sorted(n - i for i in g))
    return out


def q_fourier(q, x, L, d):
    """Q(d) = (1/N) sum_j q_j^-2 exp(i 2 pi d x_j / L) for integer offsets d."""
    q = np.asarray(q, dtype=complex)
    d = np.atleast_1d(d)
    return (np.exp(2j * np.pi * np.outer(d, x) / L) @ (q ** -2.0)) / len(q)


class AxisBands:
    """Bands, eigenvalues lambda[n] and per-band blocks X of one axis."""

    def __init__(self, axis, nbw=N_BW):
        n, L = axis.n, axis.L
        self.n = n
        self.bands = bands(n, nbw)
        self.lam = np.zeros(n, dtype=complex)
        self.X = []   # X[b][nu][m], nu and m local to band b
        self.Kl = []  # the blocks K_l themselves
        dmax = max(len(b) for b in self.bands)
        Qd = q_fourier(axis.q, axis.x, L, np.arange(-(dmax - 1), dmax))
        Q = lambda dd: Qd[dd + dmax - 1]
        for b in self.bands:
            k = axis.k[b]
            idx = np.asarray(b)
            Kl = 0.5 * np.outer(k, k) * Q(idx[None, :] - idx[:, None])
            w, V = np.linalg.eig(Kl)
            V = V / np.sqrt(np.sum(V * V, axis=0))[None, :]
            self.lam[idx] = w
            self.X.append(V.T)
            self.Kl.append(Kl)

    def apply_X(self, v, axis, transpose=False):
        """y = X v (or X^T v) along ``axis`` of a Fourier-space array."""
        v = np.moveaxis(np.asarray(v, dtype=complex), axis, -1)
        out = np.empty_like(v)
        for b, Xb in zip(self.bands, self.X):
            out[..., b] = v[..., b] @ (Xb if transpose else Xb.T)
        return np.moveaxis(out, -1, axis)


def preconditioner(op, nbw=N_BW):
    """P^-1 of Eq. PreconFFT_ECS for an ``oracle.sse.Operator`` (1D, 2D or 3D).
    Axis a of the grid is array axis nd - 1 - a (x fastest)."""
    axes = op.axes
    nd = len(axes)
    ab = [AxisBands(a, nbw) for a in axes]
    div = -op.E
    for a, bnd in enumerate(ab):
        shape = [1] * nd
        shape[nd - 1 - a] = bnd.n
        div = div + bnd.lam.reshape(shape)

    def apply(r):
        s = op._F(r)
        for a, bnd in enumerate(ab):
            s = bnd.apply_X(s, nd - 1 - a)
        s = s / div
        for a, bnd in reversed(list(enumerate(ab))):
            s = bnd.apply_X(s, nd - 1 - a, transpose=True)
        return op._Finv(s)
    return apply
