"""Pins of the learned-correction oracle (oracle.learned) against things
other than itself: FFT circular convolution, central finite differences,
Adam's closed form under a constant gradient, COCG with the plain
preconditioner and a dense solve, and the fallback on a useless
preconditioner."""
import numpy as np
import pytest

from oracle import learned as lo
from oracle import sse as os_
from oracle import tdse as ot


def _fft_conv(x, W, b):
    B, cin, H, Wd = x.shape
    cout = W.shape[1]
    X = np.fft.fft2(x)
    y = np.zeros((B, cout, H, Wd))
    for co in range(cout):
        acc = np.zeros((B, H, Wd), dtype=complex)
        for ci in range(cin):
            k = np.zeros((H, Wd))
            for t, (dy, dx) in enumerate(lo.TAPS):
                k[(-dy) % H, (-dx) % Wd] += W[t, co, ci]
            acc += X[:, ci] * np.fft.fft2(k)[None]
        y[:, co] = np.fft.ifft2(acc).real + b[co]
    return y


def test_conv_is_a_circular_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 7, 5))
    W = rng.normal(size=(9, 4, 3))
    b = rng.normal(size=4)
    assert np.allclose(lo.conv(x, W, b), _fft_conv(x, W, b), atol=1e-12)


def test_conv_backward_is_the_adjoint():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 6, 6))
    W = rng.normal(size=(9, 5, 3))
    dy = rng.normal(size=(2, 5, 6, 6))
    dW, db, dx = lo.conv_backward(x, W, dy)
    # <conv(x), dy> is linear in x and in W: its gradients are dx and dW
    lin = lambda x_, W_: np.sum(lo.conv(x_, W_, np.zeros(5)) * dy)
    ex = rng.normal(size=x.shape)
    eW = rng.normal(size=W.shape)
    assert np.isclose(lin(ex, W), np.sum(dx * ex), rtol=1e-12)
    assert np.isclose(lin(x, eW), np.sum(dW * eW), rtol=1e-12)
    assert np.allclose(db, dy.sum(axis=(0, 2, 3)))


def _tiny_batch(seed, B=2, H=6, Wd=8):
    rng = np.random.default_rng(seed)
    r = rng.normal(size=(B, H, Wd)) + 1j * rng.normal(size=(B, H, Wd))
    pz = rng.normal(size=(B, H, Wd)) + 1j * rng.normal(size=(B, H, Wd))
    e = rng.normal(size=(B, H, Wd)) + 1j * rng.normal(size=(B, H, Wd))
    s = np.sqrt(np.mean(np.abs(r) ** 2, axis=(1, 2)))
    return r, pz, e, s


def test_gradients_match_central_differences():
    r, pz, e, s = _tiny_batch(2)
    params = lo.init_params(3)
    params = [(W, np.random.default_rng(4 + i).normal(scale=0.1, size=b.shape)) for i, (W, b) in enumerate(params)]
    loss, grads = lo.loss_and_grads(params, r, pz, e, s, exact=True)
    rng = np.random.default_rng(5)
    h = 1e-6
    for li in range(3):
        for k in (0, 1):
            for _ in range(6):
                P = [list(p) for p in params]
                arr = P[li][k]
                idx = tuple(rng.integers(n) for n in arr.shape)
                plus = [tuple(q.copy() for q in p) for p in P]
                minus = [tuple(q.copy() for q in p) for p in P]
                plus[li][k][idx] += h
                minus[li][k][idx] -= h
                fd = (lo.loss_only(plus, r, pz, e, s, exact=True) - lo.loss_only(minus, r, pz, e, s, exact=True)) / (2 * h)
                an = grads[li][k][idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (li, k, idx, fd, an)


def test_rounded_network_gradient_uses_the_rounded_weights():
    r, pz, e, s = _tiny_batch(6)
    params = lo.init_params(7)
    _, g_r = lo.loss_and_grads(params, r, pz, e, s)
    rounded = [(lo.f16(W), b) for W, b in params]
    _, g_e = lo.loss_and_grads(rounded, r, pz, e, s)
    for (a, b), (c, d) in zip(g_r, g_e):
        assert np.array_equal(a, c) and np.array_equal(b, d)


def test_adam_constant_gradient_closed_form():
    params = [(np.full((9, 2, 1), 0.5), np.zeros(2))]
    grads = [(np.full((9, 2, 1), -0.3), np.full(2, 2.0))]
    state = {"t": 0, "m": {}, "v": {}}
    lr = 1e-2
    for _ in range(5):
        params = lo.adam_step(params, grads, state, lr)
    # bias-corrected moments equal g and g^2, so each step moves lr g/(|g|+eps)
    assert np.allclose(params[0][0], 0.5 + 5 * lr * 0.3 / (0.3 + 1e-8), rtol=1e-12)
    assert np.allclose(params[0][1], -5 * lr * 2.0 / (2.0 + 1e-8), rtol=1e-12)


def _small_operator(n=16, E=0.7):
    L = n * 0.4
    ax = ot.Axis(n, L, R0=0.7 * L / 2, theta=0.5)
    V = ot.softcore(1.0, 0.64, ax.x[None, :], ax.x[:, None])
    return os_.Operator((ax, ax), V, E)


def test_flexible_cocg_with_zero_network_is_cocg():
    op = _small_operator()
    rng = np.random.default_rng(8)
    f = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    zero = [(np.zeros_like(W), np.zeros_like(b)) for W, b in lo.init_params(9)]
    x1, it1, res1, fb = lo.flexible_cocg(op, f, lo.correction_preconditioner(op, zero), rtol=1e-10)
    x0, it0, res0 = os_.cocg(op, f, rtol=1e-10)
    xd = os_.dense_solve(op, f)
    assert not fb
    assert abs(it1 - it0) <= 1
    assert np.linalg.norm(x1 - xd) / np.linalg.norm(xd) < 1e-8
    assert res1 <= 1e-10


def test_flexible_cocg_falls_back_on_a_useless_preconditioner():
    op = _small_operator()
    rng = np.random.default_rng(10)
    f = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    noise = lambda r: rng.normal(size=r.shape) + 1j * rng.normal(size=r.shape)
    x, it, res, fb = lo.flexible_cocg(op, f, noise, rtol=1e-9, patience=10, maxit=5000)
    assert fb
    assert res <= 1e-9


def test_library_initial_weights_follow_the_oracle_recipe():
    # the package's seeded initial weights (input generation) and the oracle's
    # initialisation draw the same numbers in the library's parameter order
    from paper_1505_06707_amd.lp_data import flat_params, init_weights, unflat_params
    w = init_weights(7)
    assert np.array_equal(w, flat_params(lo.init_params(7)))
    back = unflat_params(w)
    for (W, b), (W0, b0) in zip(back, lo.init_params(7)):
        assert np.allclose(W, W0, rtol=1e-7) and np.array_equal(b, b0)
