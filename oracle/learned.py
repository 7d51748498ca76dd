"""A learned correction to the FFT preconditioner, in FP64 (test
infrastructure only; not from the paper).

The correction network N is three periodic 3x3 convolutions, 4 -> 16 -> 16 ->
2 channels, ReLU after the first two, applied to the residual r and the FFT
preconditioned residual P^-1 r of Sec. III (Eq. PreconFFT), both divided by
the root-mean-square s of r:

    z = P^-1 r + s N(r/s, P^-1 r/s).

Definitions fixed here (both sides implement them):
* Channels of the input x0: Re(r/s), Im(r/s), Re(P^-1 r/s), Im(P^-1 r/s),
  stored as FP16 values.  Hidden activations are stored as FP16 values; the
  output of the third layer is not rounded.  Weights are FP16 values (FP32
  master copies are what the optimiser updates).
* Layer: y[co, p] = b[co] + sum over taps t = (dy, dx) in {-1, 0, 1}^2 and
  input channels ci of W[t, co, ci] x[ci, p + (dy, dx)], indices periodic on
  the grid, tap index t = 3 (dy + 1) + (dx + 1).
* Training loss of a batch: mean over samples, pixels and the two output
  channels of (y - target)^2 with target = (e - P^-1 r)/s, e = x* - x_k the
  error of the iterate that left residual r.
* Adam (Kingma and Ba, 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and
  bias correction.
* Flexible COCG: the COCG recurrences of ``oracle.sse.cocg`` with a
  preconditioner that may vary, beta = r_{k+1}^T (z_{k+1} - z_k) / rho_k.
  When the residual has not reached a new minimum for ``patience``
  iterations, the solve continues with the plain FFT preconditioner from the
  true residual (fallback).
"""
import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
LAYERS = ((4, 16), (16, 16), (16, 2))
ADAM = dict(beta1=0.9, beta2=0.999, eps=1e-8)


def f16(a):
    """Round to FP16 values (kept as float64)."""
    return np.asarray(a, dtype=np.float64).astype(np.float16).astype(np.float64)


def init_params(seed):
    """Seeded He-style initial weights; list of (W [9, cout, cin], b [cout])."""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in LAYERS:
        W = rng.normal(scale=np.sqrt(2.0 / (9 * cin)), size=(9, cout, cin))
        out.append((W, np.zeros(cout)))
    out[-1] = (out[-1][0] * 0.1, out[-1][1])
    return out


def conv(x, W, b):
    """Periodic 3x3 convolution of x [B, cin, H, W] with W [9, cout, cin]."""
    B, cin, H, Wd = x.shape
    cout = W.shape[1]
    y = np.broadcast_to(b[None, :, None, None], (B, cout, H, Wd)).copy()
    for t, (dy, dx) in enumerate(TAPS):
        # x[ci, p + (dy, dx)]: roll by the negative shift
        xs = np.roll(x, shift=(-dy, -dx), axis=(2, 3))
        y += np.einsum("oc,bchw->bohw", W[t], xs)
    return y


def conv_backward(x, W, dy):
    """Gradients of a periodic 3x3 convolution: (dW, db, dx)."""
    dW = np.empty_like(W)
    for t, (ddy, ddx) in enumerate(TAPS):
        xs = np.roll(x, shift=(-ddy, -ddx), axis=(2, 3))
        dW[t] = np.einsum("bohw,bchw->oc", dy, xs)
    db = dy.sum(axis=(0, 2, 3))
    dx = np.zeros_like(x)
    for t, (ddy, ddx) in enumerate(TAPS):
        # y[p] uses x[p + d]: x[q] receives W^T dy[q - d]
        dx += np.roll(np.einsum("oc,bohw->bchw", W[t], dy), shift=(ddy, ddx), axis=(2, 3))
    return dW, db, dx


def features(r, pz, s, exact=False):
    """x0 [B, 4, H, W] from residuals r, P^-1 r [B, H, W] and scales s [B].
    exact=True skips the FP16 rounding (for finite-difference checks)."""
    a = r / s[:, None, None]
    c = pz / s[:, None, None]
    x = np.stack([a.real, a.imag, c.real, c.imag], axis=1)
    return x if exact else f16(x)


def forward(params, x0, exact=False):
    """Network output [B, 2, H, W] and the stored activations."""
    rnd = (lambda a: a) if exact else f16
    acts = [x0]
    x = x0
    for li, (W, b) in enumerate(params):
        y = conv(x, rnd(W), b)
        if li < len(params) - 1:
            x = rnd(np.maximum(y, 0.0))
            acts.append(x)
        else:
            x = y
    return x, acts


def loss_and_grads(params, r, pz, e, s, exact=False):
    """Loss of one batch and the gradients with respect to every W and b
    (the FP16-rounded weights are the ones differentiated)."""
    rnd = (lambda a: a) if exact else f16
    x0 = features(r, pz, s, exact)
    y, acts = forward(params, x0, exact)
    t = (e - pz) / s[:, None, None]
    T = np.stack([t.real, t.imag], axis=1)
    count = y.size
    loss = float(np.sum((y - T) ** 2) / count)
    dy = 2.0 * (y - T) / count
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        dW, db, dx = conv_backward(acts[li], rnd(W), dy)
        grads[li] = (dW, db)
        if li > 0:
            dy = dx * (acts[li] > 0)
    return loss, grads


def loss_only(params, r, pz, e, s, exact=False):
    x0 = features(r, pz, s, exact)
    y, _ = forward(params, x0, exact)
    t = (e - pz) / s[:, None, None]
    T = np.stack([t.real, t.imag], axis=1)
    return float(np.sum((y - T) ** 2) / y.size)


def adam_step(params, grads, state, lr):
    """One Adam update of every parameter (state: dict with 't', 'm', 'v')."""
    b1, b2, eps = ADAM["beta1"], ADAM["beta2"], ADAM["eps"]
    state["t"] += 1
    t = state["t"]
    out = []
    for li, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for k, (p, g) in enumerate(((W, gW), (b, gb))):
            key = (li, k)
            m = b1 * state["m"].get(key, 0.0) + (1 - b1) * g
            v = b2 * state["v"].get(key, 0.0) + (1 - b2) * g * g
            state["m"][key], state["v"][key] = m, v
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out


def correction_preconditioner(op, params):
    """z = P^-1 r + s N(r/s, P^-1 r/s) for one 2D field r."""
    def apply(r):
        pz = op.precond(r)
        s = np.sqrt(np.mean(np.abs(r) ** 2))
        if s == 0:
            return pz
        y, _ = forward(params, features(r[None], pz[None], np.array([s])))
        return pz + s * (y[0, 0] + 1j * y[0, 1])
    return apply


def flexible_cocg(op, f, precond, rtol=1e-8, maxit=10000, patience=30):
    """COCG with a variable preconditioner and the plain-preconditioner
    fallback.  Returns (x, iterations, true relative residual, fell_back)."""
    dot = lambda u, v: np.sum(u * v)
    nrm = lambda u: np.sqrt(np.sum(np.abs(u) ** 2))
    f = np.asarray(f, dtype=complex)
    fn = nrm(f)
    x = np.zeros_like(f)
    r = f.copy()
    it = 0
    fell_back = False
    M = precond
    while True:
        z = M(r)
        p = z.copy()
        rho = dot(r, z)
        best, since = np.inf, 0
        while it < maxit:
            w = op.matvec(p)
            alpha = rho / dot(p, w)
            x = x + alpha * p
            r = r - alpha * w
            it += 1
            res = nrm(r) / fn
            if res <= rtol:
                break
            if res < best:
                best, since = res, 0
            else:
                since += 1
            if not fell_back and since >= patience:
                fell_back = True
                M = op.precond
                break
            zn = M(r)
            beta = dot(r, zn - z) / rho
            rho = dot(r, zn)
            p = zn + beta * p
            z = zn
        r = f - op.matvec(x)
        true = nrm(r) / fn
        if true <= rtol or it >= maxit:
            return x, it, true, fell_back
