"""Pins of the oracle's 3D propagation (the separable reading of Sec. II for
three axes): brute force with dense matrices, the tensor product of the
(pinned) 1D steps for separable problems, the free Gaussian closed form, norm
conservation without ECS, time reversal and absorption."""
import numpy as np
import pytest

from oracle import contour, grid, tdse
from tests import closed_forms as cf


def _axis(n, L, kind=contour.SECS, R0=None, theta=0.5):
    return tdse.Axis(n, L, kind=kind, R0=R0, theta=theta)


def _dense_cn(ax, tau):
    I = np.eye(ax.n)
    C = ax.C.toarray()
    return np.linalg.solve(I + 0.5j * tau * C, I - 0.5j * tau * C)


def test_step_equals_dense_brute_force_3d():
    """Different lengths per axis, a potential that is not symmetric in the
    axes (the field along x), dense F = F_z (x) F_y (x) F_x."""
    ax, ay, az = _axis(8, 6.4, R0=2.0), _axis(6, 4.8, R0=1.5), _axis(4, 4.0, R0=1.2)
    prob = tdse.Problem3D(ax, ay, az, Zc=1.0, a2=0.64)
    tau, f = 0.05, 0.04
    F = np.kron(grid.dft_matrix(az.n, az.L), np.kron(grid.dft_matrix(ay.n, ay.L), grid.dft_matrix(ax.n, ax.L)))
    K = (ax.k[None, None, :] ** 2 + ay.k[None, :, None] ** 2 + az.k[:, None, None] ** 2).ravel() / 2
    Kh = np.diag(np.exp(-1j * K * tau / 2))
    Uh = np.diag(np.exp(-1j * prob.potential(f).ravel() * tau / 2))
    Ix, Iy, Iz = np.eye(ax.n), np.eye(ay.n), np.eye(az.n)
    CN = (np.kron(_dense_cn(az, tau), np.kron(Iy, Ix)) @ np.kron(Iz, np.kron(_dense_cn(ay, tau), Ix))
          @ np.kron(Iz, np.kron(Iy, _dense_cn(ax, tau))))
    M = F.conj().T @ Kh @ F @ Uh @ CN @ Uh @ F.conj().T @ Kh @ F
    rng = np.random.default_rng(12)
    v = rng.normal(size=(az.n, ay.n, ax.n)) + 1j * rng.normal(size=(az.n, ay.n, ax.n))
    assert np.allclose(prob.step(v, tau, f).ravel(), M @ v.ravel(), atol=1e-13)


def test_separable_problem_is_the_product_of_1d_propagations():
    """U = 0: every factor of the step acts on one axis or commutes, so a
    product state stays the product of the three 1D propagations."""
    ax, ay, az = _axis(64, 12.8, R0=4.0), _axis(32, 9.6, R0=3.0), _axis(48, 9.6, kind=contour.TFECS, R0=3.0)
    a = cf.free_gaussian(ax.x, 0.0, 1.0, 2.0)
    b = cf.free_gaussian(ay.x, 0.0, -0.5, -1.5)
    c = cf.free_gaussian(az.x, 0.0, 0.3, 1.0)
    tau, nst = 0.05, 30
    got = tdse.Problem3D(ax, ay, az, Zc=0.0).propagate(c[:, None, None] * b[None, :, None] * a[None, None, :], tau,
                                                       np.zeros(nst))
    pa = tdse.Problem1D(ax, Zc=0.0).propagate(a, tau, np.zeros(nst))
    pb = tdse.Problem1D(ay, Zc=0.0).propagate(b, tau, np.zeros(nst))
    pc = tdse.Problem1D(az, Zc=0.0).propagate(c, tau, np.zeros(nst))
    want = pc[:, None, None] * pb[None, :, None] * pa[None, None, :]
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-13
    assert np.linalg.norm(got) < 0.99 * np.linalg.norm(a) * np.linalg.norm(b) * np.linalg.norm(c)   # strips absorbed


def test_free_gaussian_matches_closed_form_3d():
    ax, ay, az = _axis(128, 51.2, R0=20.5), _axis(120, 48.0, R0=19.2), _axis(112, 44.8, R0=17.9)
    prob = tdse.Problem3D(ax, ay, az, Zc=0.0)
    X, Y, Z = ax.x[None, None, :], ay.x[None, :, None], az.x[:, None, None]
    g0 = cf.free_gaussian(X, 0.0, 0.5, 0.8) * cf.free_gaussian(Y, 0.0, -0.4, -0.6) * cf.free_gaussian(Z, 0.0, 0.2, 0.3)
    tau, nst = 0.05, 16
    got = prob.propagate(g0, tau, np.zeros(nst))
    t = tau * nst
    want = cf.free_gaussian(X, t, 0.5, 0.8) * cf.free_gaussian(Y, t, -0.4, -0.6) * cf.free_gaussian(Z, t, 0.2, 0.3)
    # h = 0.4: the spectral truncation of the k0 = 0.8 packet alone is 2.7e-12
    # in 1D on the same axis
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 5e-12


def test_norm_is_conserved_without_ecs_with_potential_and_field_3d():
    ax, ay, az = _axis(32, 12.8, kind=contour.OFF), _axis(24, 9.6, kind=contour.OFF), _axis(16, 8.0, kind=contour.OFF)
    prob = tdse.Problem3D(ax, ay, az, Zc=1.0, a2=0.64)
    X, Y, Z = ax.x[None, None, :], ay.x[None, :, None], az.x[:, None, None]
    psi0 = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / 2 + 0.3j * X)
    f = 0.05 * np.sin(0.3 * np.arange(60))
    psi = prob.propagate(psi0, 0.05, f)
    assert abs(np.linalg.norm(psi) / np.linalg.norm(psi0) - 1) < 1e-13
    assert np.linalg.norm(psi - psi0) > 0.1 * np.linalg.norm(psi0)


def test_time_reversal_3d():
    ax, ay, az = _axis(32, 12.8, R0=4.0), _axis(24, 9.6, R0=3.0), _axis(16, 6.4, R0=2.0)
    prob = tdse.Problem3D(ax, ay, az, Zc=1.0, a2=0.64)
    X, Y, Z = ax.x[None, None, :], ay.x[None, :, None], az.x[:, None, None]
    psi0 = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / 2 + 0.2j * Y)
    f = 0.04 * np.cos(0.2 * np.arange(8))
    fwd = prob.propagate(psi0, 0.05, f)
    back = prob.propagate(fwd, -0.05, f[::-1])
    assert np.linalg.norm(back - psi0) / np.linalg.norm(psi0) < 1e-11


# ---- stationary equation in 3D (Sec. III, Eq. linsys; the FFT preconditioner
# of Eq. PreconFFT with the full 3D transform)

def _op3(E, kinds=(contour.SECS, contour.SECS, contour.TFECS), Zc=1.0, n=(8, 6, 4)):
    axes = [_axis(n[0], 6.4, kind=kinds[0], R0=2.0), _axis(n[1], 4.8, kind=kinds[1], R0=1.5),
            _axis(n[2], 4.0, kind=kinds[2], R0=1.2)]
    ax, ay, az = axes
    V = tdse.softcore(Zc, 0.64, ax.z[None, None, :], ay.z[None, :, None], az.z[:, None, None])
    from oracle import sse
    return axes, sse.Operator(axes, V, E)


def test_3d_operator_is_complex_symmetric_and_cocg_matches_dense():
    from oracle import sse
    _, op = _op3(0.7)
    A = op.dense()
    assert np.allclose(A, A.T, atol=1e-13)
    assert not np.allclose(A, A.conj().T, atol=1e-6)
    rng = np.random.default_rng(13)
    f = rng.normal(size=(4, 6, 8)) + 1j * rng.normal(size=(4, 6, 8))
    x, it, res = sse.cocg(op, f, rtol=1e-13)
    xd = sse.dense_solve(op, f)
    assert res <= 1e-13
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


def test_3d_matvec_approximates_the_continuous_operator():
    """ECS off, smooth f: A f = -1/2 lap f + (U - E) f to spectral accuracy."""
    from oracle import sse
    axes = [_axis(n, 0.4 * n, kind=contour.OFF) for n in (56, 52, 48)]
    ax, ay, az = axes
    X, Y, Z = ax.x[None, None, :], ay.x[None, :, None], az.x[:, None, None]
    V = tdse.softcore(1.0, 0.64, X.astype(complex), Y.astype(complex), Z.astype(complex))
    op = sse.Operator(axes, V, 0.4)
    r2 = X ** 2 + Y ** 2 + Z ** 2
    f = np.exp(-r2 / 2)
    lap = (r2 - 3) * f
    assert np.max(np.abs(op.matvec(f) - (-0.5 * lap + (V - 0.4) * f))) < 1e-11


def test_3d_preconditioner_is_the_exact_inverse_without_ecs_and_potential():
    from oracle import sse
    _, op = _op3(0.37, kinds=(contour.OFF,) * 3, Zc=0.0)
    rng = np.random.default_rng(14)
    v = rng.normal(size=(4, 6, 8)) + 1j * rng.normal(size=(4, 6, 8))
    assert np.allclose(op.precond(op.matvec(v)), v, atol=1e-12)
    x, it, res = sse.cocg(op, v, rtol=1e-12)
    assert it == 1 and res < 1e-12
