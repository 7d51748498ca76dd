"""What a learned local correction of the FFT preconditioner (Sec. III,
Eq. PreconFFT) can gain in a form that COCG accepts: evidence from the FP64
oracle on a small grid of the stationary workload (96^2, h = 0.2, soft-core,
SECS from 80% of the half-width).

COCG needs a fixed, linear, complex-symmetric preconditioner.  The learned
network is nonlinear (ReLU) and not complex-linear, so in COCG it is used in
the flexible form, where it stagnates and falls back.  These tests fix why no
COCG-valid variant of a local, pair-trained correction can do better:

* the iteration count is set by the soft-core potential, whose effect on the
  solution is nonlocal (with U = 0 COCG needs a fraction of the iterations);
* the best translation-invariant linear correction fitted to PCG's own
  residual/error pairs (a Fourier multiplier, the least-squares optimum for
  every k) makes COCG slower, not faster;
* the best local linear correction with the network's receptive field
  (7 x 7 on the inputs r and P^-1 r), used where it cannot break COCG, as the
  initial iterate, leaves a larger residual than x0 = 0 and saves nothing;
* a diagonal rescaling by the contour, D P^-1 D with D = q(x) q(y), does not
  help either;
* the best position-dependent, complex-symmetric local correction
  M^-1 = P^-1 + S (a 3 x 3 stencil whose weights are linear in the features
  1, U, U^2 and the contour factors q^-2: the linear family a symmetric
  G^T G-type correction with position features lies in), fitted by least
  squares to PCG's pairs, predicts about 1% of e - P^-1 r and makes COCG
  diverge.
"""
import numpy as np
import pytest

from oracle import contour, grid, sse, tdse
from paper_1505_06707_amd import workloads as wl

N, H = 96, 0.2


def _problem(E, Zc=1.0):
    L = N * H
    ax = tdse.Axis(N, L, kind=contour.SECS, R0=0.8 * L / 2, theta=0.5)
    V = tdse.softcore(Zc, 0.64, ax.z[None, :], ax.z[:, None])
    return ax, sse.Operator((ax, ax), V, E)


def _cocg_from(op, f, x0, rtol=1e-8, maxit=4000):
    dot = lambda u, v: np.sum(u * v)
    nrm = lambda u: np.sqrt(np.sum(np.abs(u) ** 2))
    x = x0.copy()
    r = f - op.matvec(x)
    z = op.precond(r)
    p = z.copy()
    rho = dot(r, z)
    fn = nrm(f)
    it = 0
    while it < maxit:
        w = op.matvec(p)
        a = rho / dot(p, w)
        x = x + a * p
        r = r - a * w
        it += 1
        if nrm(r) / fn <= rtol:
            break
        z = op.precond(r)
        rn = dot(r, z)
        p = z + rn / rho * p
        rho = rn
    return it


def _pairs(op, f, keep=(0, 1, 2, 4, 8, 16, 32, 64)):
    """(r_k, e_k = x* - x_k) pairs of plain COCG on f."""
    xs, _, _ = sse.cocg(op, f, rtol=1e-12, maxit=4000)
    dot = lambda u, v: np.sum(u * v)
    x = np.zeros_like(f)
    r = f.copy()
    z = op.precond(r)
    p = z.copy()
    rho = dot(r, z)
    out = [(r.copy(), xs - x)]
    for it in range(1, max(keep) + 1):
        w = op.matvec(p)
        a = rho / dot(p, w)
        x = x + a * p
        r = r - a * w
        if it in keep:
            out.append((r.copy(), xs - x))
        z = op.precond(r)
        rn = dot(r, z)
        p = z + rn / rho * p
        rho = rn
    return out


@pytest.mark.parametrize("E", [0.1, 1.5])
def test_the_coulomb_term_sets_the_iteration_count(E):
    f = -wl.smooth_source(N, N, seed=0)
    _, op = _problem(E)
    _, op0 = _problem(E, Zc=0.0)
    full = _cocg_from(op, f, np.zeros_like(f))
    free = _cocg_from(op0, f, np.zeros_like(f))
    assert free < 0.7 * full


@pytest.mark.parametrize("E", [0.7, 1.5])
def test_a_pair_fitted_fourier_multiplier_slows_cocg(E):
    ax, op = _problem(E)
    F = lambda v: grid.forward(grid.forward(v, ax.L, axis=1), ax.L, axis=0)
    Fi = lambda v: grid.inverse(grid.inverse(v, ax.L, axis=0), ax.L, axis=1)
    num = np.zeros((N, N), complex)
    den = np.zeros((N, N))
    for seed in (101, 102, 103):
        for r, e in _pairs(op, -wl.smooth_source(N, N, seed=seed)):
            R, Ee = F(r), F(e)
            num += Ee * np.conj(R)
            den += np.abs(R) ** 2
    d = num / den
    flip = (-np.arange(N)) % N
    d = 0.5 * (d + d[flip][:, flip])            # even in k: P^-1 stays complex symmetric
    f = -wl.smooth_source(N, N, seed=0)
    plain = _cocg_from(op, f, np.zeros_like(f))
    op.precond = lambda v: Fi(d * F(v))
    fitted = _cocg_from(op, f, np.zeros_like(f))
    assert fitted > plain


@pytest.mark.parametrize("E", [0.1, 0.7, 1.5])
def test_the_best_local_linear_initial_iterate_saves_nothing(E):
    _, op = _problem(E)
    shifts = [(dy, dx) for dy in range(-3, 4) for dx in range(-3, 4)]

    def design(f, pf):
        return np.stack([np.roll(s, (-dy, -dx), axis=(0, 1)).ravel() for s in (f, pf) for dy, dx in shifts], axis=1)

    X, Y = [], []
    for seed in range(101, 107):
        f = -wl.smooth_source(N, N, seed=seed)
        xs, _, _ = sse.cocg(op, f, rtol=1e-11, maxit=4000)
        pf = op.precond(f)
        X.append(design(f, pf))
        Y.append((xs - pf).ravel())
    coef, *_ = np.linalg.lstsq(np.concatenate(X), np.concatenate(Y), rcond=None)
    f = -wl.smooth_source(N, N, seed=0)
    pf = op.precond(f)
    x0 = pf + (design(f, pf) @ coef).reshape(N, N)
    assert np.linalg.norm(f - op.matvec(x0)) > np.linalg.norm(f)
    assert _cocg_from(op, f, x0) >= _cocg_from(op, f, np.zeros_like(f)) - 1


def test_rescaling_by_the_contour_does_not_help():
    ax, op = _problem(0.7)
    f = -wl.smooth_source(N, N, seed=0)
    plain = _cocg_from(op, f, np.zeros_like(f))
    D = ax.q[None, :] * ax.q[:, None]
    P = op.precond
    op.precond = lambda v: D * P(D * v)
    assert _cocg_from(op, f, np.zeros_like(f)) >= plain


def test_the_best_symmetric_position_dependent_local_correction_explains_nothing():
    """S = sum_d (D_d T_d + T_-d D_d), (T_d v)(x) = v(x + d), d over the half
    of a 3 x 3 stencil, D_d = sum_j c_dj phi_j with phi = 1, U, U^2,
    q_x^-2 + q_y^-2, (q_x^-2 - 1)(q_y^-2 - 1): complex symmetric for every c,
    so COCG accepts P^-1 + S.  The least-squares c over PCG's (r_k, e_k) pairs
    of four training sources leaves >= 95% of e - P^-1 r unexplained, and
    COCG with P^-1 + S needs more iterations than with P^-1 on a held-out
    source."""
    E = 0.7
    ax, op = _problem(E)
    V = op.V
    iq = 1 / ax.q ** 2
    feats = [np.ones((N, N), complex), V, V ** 2, iq[None, :] + iq[:, None], (iq[None, :] - 1) * (iq[:, None] - 1)]
    offs = [(dy, dx) for dy in range(-1, 2) for dx in range(-1, 2) if (dy, dx) >= (0, 0)]
    T = lambda v, d: np.roll(v, (-d[0], -d[1]), axis=(0, 1))

    def columns(v):
        cols = []
        for d in offs:
            for ph in feats:
                cols.append(2 * ph * v if d == (0, 0) else ph * T(v, d) + T(ph * v, (-d[0], -d[1])))
        return np.stack([c.ravel() for c in cols], axis=1)

    X, Y = [], []
    for seed in (101, 102, 103, 104):
        for r, e in _pairs(op, -wl.smooth_source(N, N, seed=seed)):
            X.append(columns(r))
            Y.append((e - op.precond(r)).ravel())
    X, Y = np.concatenate(X), np.concatenate(Y)
    coef, *_ = np.linalg.lstsq(X, Y, rcond=None)
    assert np.linalg.norm(X @ coef - Y) / np.linalg.norm(Y) > 0.95
    S = lambda v: (columns(v) @ coef).reshape(N, N)
    rng = np.random.default_rng(0)
    u, w = (rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N)) for _ in range(2))
    assert abs(np.sum(u * S(w)) - np.sum(w * S(u))) <= 1e-12 * abs(np.sum(u * S(w)))   # S = S^T
    f = -wl.smooth_source(N, N, seed=0)
    plain = _cocg_from(op, f, np.zeros_like(f))
    P = op.precond
    op.precond = lambda v: P(v) + S(v)
    assert _cocg_from(op, f, np.zeros_like(f), maxit=3 * plain) > plain
