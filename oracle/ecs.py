"""Three-point ECS kinetic operator, remainder C and Crank-Nicolson
(Sec. II, Eqs. Ks_FD, K_FD, C_FD and the CN formula).  Test infrastructure.

Readings:
* Boundary condition of the three-point stencils: periodic, like the Fourier
  basis, so the two scaled regions at the box edges are joined through the
  boundary (the paper's own picture of them as stitched together, Sec. III).
  The stencil between node N-1 and node 0 uses q at the box edge, q(b) = q(a).
* q^{-1/2} takes the principal branch.
* Where q is infinite (TFECS at the box edge), 1/q = 0: the stencil does not
  couple through that cell edge.
* C = K_s - K_FD is exactly zero on rows whose node and both neighbouring
  cell edges have q = 1 (Sec. II: C vanishes where q = 1), so C is a cyclic
  tridiagonal matrix that is non-zero only on the scaled strip.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _neighbours(n):
    j = np.arange(n)
    return (j + 1) % n, (j - 1) % n


def _over(a, q):
    """a / q, and 0 where q is infinite (the TFECS contour at the box edge)."""
    inf = np.isinf(q.real) | np.isinf(q.imag)
    safe = np.where(inf, 1.0, q)
    return np.where(inf, 0.0, a / safe)


def apply_Ks(psi, q, qm, h):
    """[K_s psi]_i of Sec. II Eq. Ks_FD, literally, with periodic indices.

    q[j] = q(x_j); qm[j] = q(x_{j+1/2}), so q_{j-1/2} = qm[j-1]."""
    n = len(q)
    jp, jm = _neighbours(n)
    qs = q ** -0.5
    fwd = _over(qs[jp] * psi[jp] - qs * psi, qm) / h
    bwd = _over(qs * psi - qs[jm] * psi[jm], qm[jm]) / h
    return -0.5 * qs / h * (fwd - bwd)


def apply_KFD(psi, h):
    """[K_FD psi]_i of Sec. II Eq. K_FD with periodic indices."""
    n = len(psi)
    jp, jm = _neighbours(n)
    return -0.5 * (psi[jp] - 2 * psi + psi[jm]) / h**2


def remainder_matrix(q, qm, h):
    """C = K_s - K_FD (Sec. II Eq. C_FD) as a sparse cyclic tridiagonal matrix.

    Entries read off Eq. Ks_FD:
      (K_s)_{j,j+1} = -(1/2h^2) q_j^{-1/2} q_{j+1}^{-1/2} / q_{j+1/2}
      (K_s)_{j,j}   =  (1/2h^2) q_j^{-1} (1/q_{j+1/2} + 1/q_{j-1/2})
    and from Eq. K_FD: off-diagonal -1/(2h^2), diagonal 1/h^2."""
    n = len(q)
    jp, jm = _neighbours(n)
    qs = q ** -0.5
    c = 1.0 / (2 * h * h)
    up = -_over(c * qs * qs[jp], qm) + c            # C_{j,j+1}
    dn = -_over(c * qs * qs[jm], qm[jm]) + c        # C_{j,j-1}
    dg = c * (1.0 / q) * (_over(1.0, qm) + _over(1.0, qm[jm])) - 2 * c
    j = np.arange(n)
    rows = np.concatenate([j, j, j])
    cols = np.concatenate([j, jp, jm])
    vals = np.concatenate([dg, up, dn])
    keep = vals != 0
    return sp.csc_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n))


class CrankNicolson:
    """exp(-i C tau) ~ (1 + i tau C/2)^-1 (1 - i tau C/2) (Sec. II, CN formula),
    applied with a sparse LU of (1 + i tau C/2)."""

    def __init__(self, C, tau):
        n = C.shape[0]
        eye = sp.identity(n, dtype=complex, format="csc")
        self.minus = (eye - 0.5j * tau * C).tocsc()
        self.lu = spla.splu((eye + 0.5j * tau * C).tocsc())

    def apply(self, v, axis=-1):
        """Apply along ``axis`` of an array (every other index is a separate
        right-hand side)."""
        v = np.moveaxis(np.asarray(v, dtype=complex), axis, 0)
        shape = v.shape
        flat = v.reshape(shape[0], -1)
        out = self.lu.solve(np.asarray(self.minus @ flat))
        return np.moveaxis(out.reshape(shape), 0, axis)
