"""Training pairs for the learned preconditioner correction.

A pair is (r_k, e_k): the residual f - A x_k left by k iterations of the plain
FFT-preconditioned COCG (Sec. III) and the error e_k = x* - x_k of that
iterate, with x* the solution to a tight tolerance.  Every solve and matrix
application runs in libsofft; torch only holds the device arrays and forms
the two differences."""
import numpy as np


def make_pairs(plan, sources, energies, schedule=(1, 2, 4, 8, 16, 32, 64), rtol_star=1e-11):
    """Pairs for every (source, energy) and every k in schedule.

    sources: complex128 device tensors [ny][nx]; returns (r, e, E) with r and e
    complex128 device tensors [npairs][ny][nx] and E a numpy array."""
    import torch
    rs, es, Es = [], [], []
    iters = 0
    for f in sources:
        for E in energies:
            xs, st, _ = plan.sse_solve(f, [E], rtol=rtol_star, maxit=20000)
            iters += st[0]["iterations"]
            for k in schedule:
                xk, _, _ = plan.sse_solve(f, [E], rtol=1e-300, maxit=int(k))
                iters += int(k)
                Ax = plan.sse_apply(0, xk[0], E)
                rs.append(f - Ax)
                es.append(xs[0] - xk[0])
                Es.append(E)
    return torch.stack(rs), torch.stack(es), np.array(Es), iters


def init_weights(seed, layers=((4, 16), (16, 16), (16, 2))):
    """Seeded initial parameters as one float32 vector in the library's order:
    He-normal weights (std sqrt(2 / (9 cin))), the output layer scaled by 0.1,
    zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (cin, cout) in enumerate(layers):
        W = rng.normal(scale=np.sqrt(2.0 / (9 * cin)), size=(9, cout, cin))
        if li == len(layers) - 1:
            W = W * 0.1
        parts += [W.ravel(), np.zeros(cout)]
    return np.concatenate(parts).astype(np.float32)


def flat_params(params):
    """Oracle-layout parameters [(W [9, cout, cin], b [cout]) x 3] as one
    float32 vector in the library's order."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unflat_params(w, layers=((4, 16), (16, 16), (16, 2))):
    out, o = [], 0
    for cin, cout in layers:
        W = np.asarray(w[o:o + 9 * cout * cin], dtype=np.float64).reshape(9, cout, cin)
        o += 9 * cout * cin
        b = np.asarray(w[o:o + cout], dtype=np.float64)
        o += cout
        out.append((W, b))
    return out
