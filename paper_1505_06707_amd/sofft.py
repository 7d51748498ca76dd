"""Thin ctypes binding of libsofft (C ABI in include/sofft.h).

Arguments are marshalled from torch device tensors (pointers, sizes) and the
current torch stream; every step of the computation runs in the HIP library.
There is no fallback: if the library is missing or the tensors are not on a
GPU, the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsofft.so")

C128, C64 = 0, 1
SECS, SHARP, ECS_OFF, TFECS = 0, 1, 2, 3
ABSORBER_CAP, ABSORBER_TFAP = 0, 1

_STATUS = {0: "SOFFT_OK", -1: "SOFFT_EINVAL", -2: "SOFFT_EUNSUPPORTED", -3: "SOFFT_EHIP",
           -4: "SOFFT_ENOMEM", -5: "SOFFT_EWORKSPACE", 1: "SOFFT_NOT_CONVERGED", 2: "SOFFT_BREAKDOWN"}


class SofftError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class SolveStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("fell_back", ctypes.c_int32),
        ("rel_residual", ctypes.c_double),
    ]


class Problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("L", ctypes.c_double * 3),
        ("R0", ctypes.c_double * 3),
        ("theta", ctypes.c_double),
        ("contour", ctypes.c_int32),
        ("charge", ctypes.c_double),
        ("a2", ctypes.c_double),
    ]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "sofft_last_error": (ctypes.c_char_p, []),
    "sofft_version": (ctypes.c_int32, []),
    "sofft_plan_create": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_void_p)]),
    "sofft_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sofft_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "sofft_plan_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "sofft_grid_nodes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "sofft_strip_length": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "sofft_propagate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_propagate_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                                              ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_norm2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_void_p]),
    "sofft_set_potential": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_make_softcore": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "sofft_add_absorber": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "sofft_sse_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_sse_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_void_p]),
    "sofft_sse_solve_shifted": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
                                               ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_sse_apply_shifted": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]),
    "sofft_sse_solve_banded": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_double,
                                              ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_sse_apply_banded": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_void_p]),
    "sofft_band_tables": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_sse_tune_shift": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "sofft_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sofft_batch_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "sofft_batch_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "sofft_batch_propagate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_batch_set_graph_steps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sofft_batch_set_launch_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.c_int32, ctypes.c_int32]),
    "sofft_batch_launch_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "sofft_lp_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p)]),
    "sofft_lp_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sofft_lp_param_count": (ctypes.c_int32, []),
    "sofft_lp_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                               ctypes.POINTER(ctypes.c_int64)]),
    "sofft_lp_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "sofft_lp_set_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_lp_get_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_lp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_lp_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "sofft_lp_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_lp_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    "sofft_sse_solve_learned": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
                                               ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "sofft_timing_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sofft_timing_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]),
}

KERNEL_ROW, KERNEL_COL, KERNEL_1D = 0, 1, 2
KERNEL_SSE_ROW_MV, KERNEL_SSE_COL_MV, KERNEL_SSE_ROW_UPD, KERNEL_SSE_COL_PREC, KERNEL_SSE_ROW_PREC = 3, 4, 5, 6, 7
KERNEL_3D_KINETIC, KERNEL_3D_STRIP = 8, 9
KERNEL_SSE_1D = 10


def exported_symbols():
    """Names the binding expects the library to export."""
    return list(_SIGS)


def lib():
    """Load libsofft.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code < 0:
        raise SofftError(code, lib().sofft_last_error().decode())
    return code


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def device_workspace(nbytes, device="cuda"):
    """A caller-owned device workspace of at least nbytes bytes, 256-byte
    aligned: (the torch tensor that owns it, aligned pointer)."""
    import torch
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    ptr = (t.data_ptr() + 255) // 256 * 256
    return t, ptr


class Plan:
    """A libsofft plan: grid, contour and potential of Sec. II, on the current device."""

    def __init__(self, n, L, R0=None, theta=0.5, contour=SECS, charge=1.0, a2=2.0, dtype=C128):
        n = list(n) if isinstance(n, (list, tuple)) else [n]
        L = list(L) if isinstance(L, (list, tuple)) else [L] * len(n)
        if R0 is None:
            R0 = [l / 2 * 0.8 for l in L]
        R0 = list(R0) if isinstance(R0, (list, tuple)) else [R0] * len(n)
        p = Problem()
        p.ndim = len(n)
        p.dtype = dtype
        for d in range(len(n)):
            p.n[d] = int(n[d])
            p.L[d] = float(L[d])
            p.R0[d] = float(R0[d])
        p.theta = float(theta)
        p.contour = int(contour)
        p.charge = float(charge)
        p.a2 = float(a2)
        self.problem = p
        self.shape = tuple(int(v) for v in reversed(n))   # [ny][nx]
        self.dtype = dtype
        h = ctypes.c_void_p()
        _check(lib().sofft_plan_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._ws = None
        self._ws_energies = -1
        self.ensure_workspace(0)

    def workspace_size(self, n_energies=0):
        """Bytes of device workspace for propagation and solves of n_energies energies."""
        b = ctypes.c_int64()
        _check(lib().sofft_workspace_size(self._h, int(n_energies), ctypes.byref(b)))
        return b.value

    def ensure_workspace(self, n_energies=0):
        """Allocate (with torch) and bind a workspace large enough for
        n_energies energies, if the bound one is smaller."""
        if n_energies <= self._ws_energies:
            return
        nbytes = self.workspace_size(n_energies)
        if self._ws is not None:
            import torch
            torch.cuda.current_stream().synchronize()   # work on the old workspace has finished
            _check(lib().sofft_plan_bind(self._h, ctypes.c_void_p(0), 0))
            self._ws = None
        t, ptr = device_workspace(nbytes)
        _check(lib().sofft_plan_bind(self._h, ctypes.c_void_p(ptr), nbytes))
        self._ws = t
        self._ws_energies = int(n_energies)

    @property
    def numel(self):
        return int(np.prod(self.shape))

    @property
    def torch_dtype(self):
        import torch
        return torch.complex128 if self.dtype == C128 else torch.complex64

    def close(self):
        if getattr(self, "_h", None):
            lib().sofft_plan_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nodes(self, axis=0):
        n = self.problem.n[axis]
        out = np.empty(n, dtype=np.float64)
        _check(lib().sofft_grid_nodes(self._h, axis, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def strip_length(self, axis=0):
        m = ctypes.c_int64()
        _check(lib().sofft_strip_length(self._h, axis, ctypes.byref(m)))
        return m.value

    def propagate(self, psi, dt, nsteps, f_mid=None, stream=None):
        """Advance psi (device tensor, in place) by nsteps steps of dt."""
        import torch
        ptr = _dev_ptr(psi, self.torch_dtype, self.numel, "psi")
        fptr = ctypes.c_void_p(0) if f_mid is None else _dev_ptr(f_mid, torch.float64, nsteps, "f_mid")
        _check(lib().sofft_propagate(self._h, ptr, float(dt), int(nsteps), fptr, _stream(stream)))
        return psi

    def set_potential(self, V0=None, W=None):
        """U = V0 + f(t) W on the grid (device tensors [ny][nx]: V0 complex128 at
        z(x), W float64); None keeps the problem's soft-core V0 / W = x.  The
        plan holds references to both, as the library reads them in place."""
        import torch
        v0 = ctypes.c_void_p(0) if V0 is None else _dev_ptr(V0, torch.complex128, self.numel, "V0")
        w = ctypes.c_void_p(0) if W is None else _dev_ptr(W, torch.float64, self.numel, "W")
        _check(lib().sofft_set_potential(self._h, v0, w))
        self._user_potential = (V0, W)

    def make_softcore(self, charge=1.0, a2=2.0, out=None, stream=None):
        """V0 = -charge / sqrt(sum z^2 + a2) on the grid (complex128 device tensor)."""
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.complex128, device="cuda")
        ptr = _dev_ptr(out, torch.complex128, self.numel, "out")
        _check(lib().sofft_make_softcore(self._h, float(charge), float(a2), ptr, _stream(stream)))
        return out

    def add_absorber(self, kind, param, v0, stream=None):
        """Add the absorbing potential ``kind`` ("cap": param = E_cap, or
        "tfap": param = k_min) of Sec. IV to the complex128 device tensor v0
        on the plan's grid, in place; returns v0."""
        import torch
        code = {"cap": ABSORBER_CAP, "tfap": ABSORBER_TFAP}[kind]
        ptr = _dev_ptr(v0, torch.complex128, self.numel, "v0")
        _check(lib().sofft_add_absorber(self._h, code, float(param), ptr, _stream(stream)))
        return v0

    def timing(self, enable=True):
        """Enable (clearing the record) or disable per-launch event timing."""
        _check(lib().sofft_timing_enable(self._h, 1 if enable else 0))

    def timing_read(self, kernel):
        """(total milliseconds, launches) of one kernel kind since enabling."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(lib().sofft_timing_read(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def sse_apply(self, op, v, E, field=0.0, out=None, stream=None, eta=0.0, banded=False):
        """w = A v (op 0) or w = P^-1 v (op 1) at energy E (device tensors);
        eta != 0 shifts the preconditioner's divisor to K - E - i eta; banded
        selects the preconditioner of Eq. PreconFFT_ECS."""
        import torch
        self.ensure_workspace(1)
        ptr = _dev_ptr(v, torch.complex128, self.numel, "v")
        if out is None:
            out = torch.empty_like(v)
        optr = _dev_ptr(out, torch.complex128, self.numel, "out")
        if banded:
            _check(lib().sofft_sse_apply_banded(self._h, int(op), ptr, optr, float(E), float(field), _stream(stream)))
        elif eta:
            _check(lib().sofft_sse_apply_shifted(self._h, int(op), ptr, optr, float(E), float(eta), float(field),
                                                 _stream(stream)))
        else:
            _check(lib().sofft_sse_apply(self._h, int(op), ptr, optr, float(E), float(field), _stream(stream)))
        return out

    def sse_solve(self, f, energies, field=0.0, rtol=1e-8, maxit=10000, out=None, stream=None, eta=None,
                  banded=False):
        """Solve (H - E_j) x_j = f for every energy; returns (x, stats, status).

        f: complex128 device tensor of the grid's shape, self.shape ([nx],
        [ny][nx] or [nz][ny][nx]), shared by all energies, or [nE] + that shape.
        eta: None (the preconditioner of Eq. PreconFFT) or per-energy shifts of
        its divisor (sofft_sse_solve_shifted).  banded: the preconditioner of
        Eq. PreconFFT_ECS (sofft_sse_solve_banded)."""
        import torch
        E = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).ravel())
        nE = len(E)
        self.ensure_workspace(nE)
        per = 1 if f.numel() == nE * self.numel and nE > 1 else 0
        fptr = _dev_ptr(f, torch.complex128, self.numel * (nE if per else 1), "f")
        if out is None:
            out = torch.empty((nE,) + self.shape, dtype=torch.complex128, device=f.device)
        optr = _dev_ptr(out, torch.complex128, nE * self.numel, "out")
        stats = (SolveStats * nE)()
        if banded:
            code = lib().sofft_sse_solve_banded(self._h, fptr, per, E.ctypes.data_as(ctypes.c_void_p), nE,
                                                float(field), optr, float(rtol), int(maxit), stats, _stream(stream))
        elif eta is None:
            code = lib().sofft_sse_solve(self._h, fptr, per, E.ctypes.data_as(ctypes.c_void_p), nE, float(field),
                                         optr, float(rtol), int(maxit), stats, _stream(stream))
        else:
            sh = np.ascontiguousarray(np.broadcast_to(np.asarray(eta, dtype=np.float64), (nE,)))
            code = lib().sofft_sse_solve_shifted(self._h, fptr, per, E.ctypes.data_as(ctypes.c_void_p),
                                                 sh.ctypes.data_as(ctypes.c_void_p), nE, float(field), optr,
                                                 float(rtol), int(maxit), stats, _stream(stream))
        _check(code)
        rows = [dict(iterations=s.iterations, status=s.status, restarts=s.restarts,
                     rel_residual=s.rel_residual) for s in stats]
        return out, rows, code

    def sse_tune_shift(self, f, energies, candidates, probe_iters=24, rtol=1e-8, field=0.0, stream=None):
        """Per-energy divisor shift chosen from the candidates by short batched
        solves (sofft_sse_tune_shift); f is one right-hand side [ny][nx]."""
        import torch
        E = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).ravel())
        cand = np.ascontiguousarray(np.asarray(candidates, dtype=np.float64).ravel())
        nE, nc = len(E), len(cand)
        self.ensure_workspace(nE * nc)
        fptr = _dev_ptr(f, torch.complex128, self.numel, "f")
        scratch = torch.empty((nE * nc,) + self.shape, dtype=torch.complex128, device=f.device)
        sptr = _dev_ptr(scratch, torch.complex128, nE * nc * self.numel, "scratch")
        out = np.zeros(nE, dtype=np.float64)
        _check(lib().sofft_sse_tune_shift(self._h, fptr, E.ctypes.data_as(ctypes.c_void_p), nE, float(field),
                                          cand.ctypes.data_as(ctypes.c_void_p), nc, int(probe_iters), float(rtol),
                                          sptr, out.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        del scratch
        return out

    def sse_solve_learned(self, lp, f, energies, field=0.0, rtol=1e-8, maxit=10000, patience=30, out=None,
                          stream=None):
        """sse_solve with the learned correction in flexible COCG; returns
        (x, stats, status), stats rows also carrying 'fell_back'."""
        import torch
        E = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).ravel())
        nE = len(E)
        self.ensure_workspace(nE)
        lp.ensure_workspace(self.shape[0], self.shape[1], nE)
        per = 1 if f.numel() == nE * self.numel and nE > 1 else 0
        fptr = _dev_ptr(f, torch.complex128, self.numel * (nE if per else 1), "f")
        if out is None:
            out = torch.empty((nE,) + self.shape, dtype=torch.complex128, device=f.device)
        optr = _dev_ptr(out, torch.complex128, nE * self.numel, "out")
        stats = (SolveStats * nE)()
        code = lib().sofft_sse_solve_learned(self._h, lp._h, fptr, per, E.ctypes.data_as(ctypes.c_void_p), nE,
                                             float(field), optr, float(rtol), int(maxit), int(patience), stats,
                                             _stream(stream))
        _check(code)
        rows = [dict(iterations=s.iterations, status=s.status, restarts=s.restarts, fell_back=s.fell_back,
                     rel_residual=s.rel_residual) for s in stats]
        return out, rows, code

    def norm2(self, psi, stream=None):
        ptr = _dev_ptr(psi, self.torch_dtype, self.numel, "psi")
        out = ctypes.c_double()
        _check(lib().sofft_norm2(self._h, ptr, ctypes.byref(out), _stream(stream)))
        return out.value


BAND_MAX = 19


def band_tables(prob, axis=0):
    """Host tables of the banded ECS eigen-preconditioner for one axis of a
    problem (sofft_band_tables): (lambda [n], X rows [n][19], start [n], width [n])."""
    n = int(prob.n[axis])
    lam = np.zeros(2 * n, dtype=np.float64)
    xr = np.zeros(2 * n * BAND_MAX, dtype=np.float64)
    st = np.zeros(n, dtype=np.int32)
    wd = np.zeros(n, dtype=np.int32)
    _check(lib().sofft_band_tables(ctypes.byref(prob), int(axis), lam.ctypes.data_as(ctypes.c_void_p),
                                   xr.ctypes.data_as(ctypes.c_void_p), st.ctypes.data_as(ctypes.c_void_p),
                                   wd.ctypes.data_as(ctypes.c_void_p)))
    return lam.view(np.complex128), xr.view(np.complex128).reshape(n, BAND_MAX), st, wd


def problem(n, L, R0=None, theta=0.5, contour=SECS, charge=1.0, a2=2.0, dtype=C128):
    """A sofft_problem structure (the arguments of Plan)."""
    n = list(n) if isinstance(n, (list, tuple)) else [n]
    L = list(L) if isinstance(L, (list, tuple)) else [L] * len(n)
    if R0 is None:
        R0 = [l / 2 * 0.8 for l in L]
    R0 = list(R0) if isinstance(R0, (list, tuple)) else [R0] * len(n)
    p = Problem()
    p.ndim = len(n)
    p.dtype = dtype
    for d in range(len(n)):
        p.n[d] = int(n[d])
        p.L[d] = float(L[d])
        p.R0[d] = float(R0[d])
    p.theta = float(theta)
    p.contour = int(contour)
    p.charge = float(charge)
    p.a2 = float(a2)
    return p


class Batch:
    """Many 2D propagations of uneven size advanced together (sofft_batch_*).

    problems: list of Problem structures (see problem()), all 2D, one dtype."""

    def __init__(self, problems):
        arr = (Problem * len(problems))(*problems)
        h = ctypes.c_void_p()
        _check(lib().sofft_batch_create(ctypes.cast(arr, ctypes.c_void_p), len(problems), ctypes.byref(h)))
        self._h = h
        self.problems = list(problems)
        self.dtype = problems[0].dtype
        b = ctypes.c_int64()
        _check(lib().sofft_batch_workspace_size(self._h, ctypes.byref(b)))
        self._ws, ptr = device_workspace(b.value)
        _check(lib().sofft_batch_bind(self._h, ctypes.c_void_p(ptr), b.value))

    def close(self):
        if getattr(self, "_h", None):
            lib().sofft_batch_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self, r):
        p = self.problems[r]
        return (int(p.n[1]), int(p.n[0]))

    def propagate(self, states, dt, nsteps, f_mid=None, norms=True, stream=None):
        """Advance every state (list of device tensors, in place); returns the
        FP64 squared norms (numpy array) when norms is true.

        f_mid: float64 device tensor [nrun][nsteps] or None."""
        import torch
        if len(states) != len(self.problems):
            raise ValueError("one state per run is needed")
        tdt = torch.complex128 if self.dtype == C128 else torch.complex64
        ptrs = (ctypes.c_void_p * len(states))()
        for r, t in enumerate(states):
            ny, nx = self.shape(r)
            ptrs[r] = _dev_ptr(t, tdt, ny * nx, f"state {r}").value
        fptr = ctypes.c_void_p(0) if f_mid is None else _dev_ptr(f_mid, torch.float64, len(states) * nsteps, "f_mid")
        out = np.zeros(len(states), dtype=np.float64)
        optr = out.ctypes.data_as(ctypes.c_void_p) if norms else ctypes.c_void_p(0)
        _check(lib().sofft_batch_propagate(self._h, ctypes.cast(ptrs, ctypes.c_void_p), float(dt), int(nsteps),
                                           fptr, optr, _stream(stream)))
        return out if norms else None

    def set_graph_steps(self, steps):
        _check(lib().sofft_batch_set_graph_steps(self._h, int(steps)))

    def set_launch_shape(self, run, pass_, threads, grid):
        _check(lib().sofft_batch_set_launch_shape(self._h, int(run), int(pass_), int(threads), int(grid)))

    def launch_shape(self, run, pass_):
        t = ctypes.c_int32()
        g = ctypes.c_int32()
        _check(lib().sofft_batch_launch_shape(self._h, int(run), int(pass_), ctypes.byref(t), ctypes.byref(g)))
        return t.value, g.value


class LearnedCorrection:
    """The correction network of sofft_lp_* (weights as one FP32 vector in the
    layout of include/sofft.h)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().sofft_lp_create(ctypes.byref(h)))
        self._h = h
        self.nparams = int(lib().sofft_lp_param_count())
        self._ws = None
        self._ws_bytes = 0

    def ensure_workspace(self, ny, nx, batch, npairs=0):
        """Allocate (with torch) and bind a workspace for calls on `batch`
        items of ny x nx that may train on npairs pairs, if the bound one is
        smaller."""
        b = ctypes.c_int64()
        _check(lib().sofft_lp_workspace_size(int(ny), int(nx), int(batch), int(npairs), ctypes.byref(b)))
        if b.value <= self._ws_bytes:
            return
        if self._ws is not None:
            import torch
            torch.cuda.current_stream().synchronize()
            _check(lib().sofft_lp_bind(self._h, ctypes.c_void_p(0), 0))
        self._ws, ptr = device_workspace(b.value)
        _check(lib().sofft_lp_bind(self._h, ctypes.c_void_p(ptr), b.value))
        self._ws_bytes = b.value

    def close(self):
        if getattr(self, "_h", None):
            lib().sofft_lp_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float32).ravel())
        if w.size != self.nparams:
            raise ValueError(f"{self.nparams} parameters expected, got {w.size}")
        _check(lib().sofft_lp_set_weights(self._h, w.ctypes.data_as(ctypes.c_void_p)))

    def get_weights(self):
        w = np.empty(self.nparams, dtype=np.float32)
        _check(lib().sofft_lp_get_weights(self._h, w.ctypes.data_as(ctypes.c_void_p)))
        return w

    def forward(self, r, pz, stream=None):
        """N's output [B][ny][nx][2] (float32 device tensor) for complex128 r, pz [B][ny][nx]."""
        import torch
        B, ny, nx = r.shape
        self.ensure_workspace(ny, nx, B)
        out = torch.empty((B, ny, nx, 2), dtype=torch.float32, device=r.device)
        _check(lib().sofft_lp_forward(self._h, _dev_ptr(r, torch.complex128, r.numel(), "r"),
                                      _dev_ptr(pz, torch.complex128, r.numel(), "pz"), ny, nx, B,
                                      _dev_ptr(out, torch.float32, out.numel(), "out"), _stream(stream)))
        return out

    def loss_grad(self, r, pz, e, stream=None):
        """(loss, gradient as a numpy float32 vector) of one batch."""
        import torch
        B, ny, nx = r.shape
        self.ensure_workspace(ny, nx, B)
        g = torch.empty(self.nparams, dtype=torch.float32, device=r.device)
        loss = ctypes.c_double()
        _check(lib().sofft_lp_loss_grad(self._h, _dev_ptr(r, torch.complex128, r.numel(), "r"),
                                        _dev_ptr(pz, torch.complex128, r.numel(), "pz"),
                                        _dev_ptr(e, torch.complex128, r.numel(), "e"), ny, nx, B,
                                        _dev_ptr(g, torch.float32, g.numel(), "grad"), ctypes.byref(loss),
                                        _stream(stream)))
        return loss.value, g.cpu().numpy()

    def backward(self, r, pz, dout, stream=None):
        """(din [B][ny][nx][4], dw [param_count]) float32 device tensors for
        dL/dN = dout [B][ny][nx][2] at inputs r, pz [B][ny][nx] (complex128)."""
        import torch
        B, ny, nx = r.shape
        self.ensure_workspace(ny, nx, B)
        din = torch.empty((B, ny, nx, 4), dtype=torch.float32, device=r.device)
        dw = torch.empty(self.nparams, dtype=torch.float32, device=r.device)
        _check(lib().sofft_lp_backward(self._h, _dev_ptr(r, torch.complex128, r.numel(), "r"),
                                       _dev_ptr(pz, torch.complex128, r.numel(), "pz"),
                                       _dev_ptr(dout, torch.float32, B * ny * nx * 2, "dout"), ny, nx, B,
                                       _dev_ptr(din, torch.float32, din.numel(), "din"),
                                       _dev_ptr(dw, torch.float32, dw.numel(), "dw"), _stream(stream)))
        return din, dw

    def train(self, plan, r, e, energies, epochs, batch, lr=1e-3, seed=0, stream=None):
        """Train on (r_k, e_k) pairs [npairs][ny][nx] of the plan's grid; returns the per-epoch losses."""
        import torch
        E = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).ravel())
        n = r.shape[0]
        if len(E) != n:
            raise ValueError("one energy per pair is needed")
        losses = np.zeros(epochs, dtype=np.float64)
        plan.ensure_workspace(1)
        self.ensure_workspace(r.shape[1], r.shape[2], int(batch), n)
        _check(lib().sofft_lp_train(self._h, plan._h, _dev_ptr(r, torch.complex128, r.numel(), "r"),
                                    _dev_ptr(e, torch.complex128, r.numel(), "e"),
                                    E.ctypes.data_as(ctypes.c_void_p), n, int(epochs), int(batch), float(lr),
                                    int(seed), losses.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return losses
