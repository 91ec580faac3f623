"""Thin Python binding of libhinv (C ABI in include/hinv.h).

Argument marshalling only: every computation runs in the HIP library.  Device
buffers are torch CUDA float64 tensors; a multivector of c columns is a tensor
of shape (c, ld) whose rows are the columns (column-major with leading
dimension ld = tensor.stride(0)).  The library must be built first
(``python -m paper_1909_03948_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhinv.so")

HINV_OK, HINV_EINVAL, HINV_ENOMEM, HINV_EHIP = 0, -1, -2, -3
HINV_ENOCONV, HINV_ESTATE, HINV_ENEGEIG, HINV_EBREAK = -4, -5, -6, -7
HESS_FULL, HESS_MISFIT, HESS_GN_FULL, HESS_GN_MISFIT = 0, 1, 2, 3
PREC_FP64, PREC_FP32_IR, PREC_AUTO = 0, 1, 2
TPROD_FP64, TPROD_BF16 = 0, 1
NEWTON_MAXREC = 64


class FcgInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("fallback", C.c_int),
                ("fallback_iterations", C.c_int), ("relres", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ProblemDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("gamma", C.c_double), ("delta", C.c_double),
                ("beta", C.c_double), ("m_prior", C.c_double), ("q", C.c_int),
                ("obs_xy", C.POINTER(C.c_double)), ("d_obs", C.POINTER(C.c_double)),
                ("sigma", C.c_double), ("precision", C.c_int), ("rtol", C.c_double),
                ("max_iter", C.c_int), ("theta1", C.c_double), ("theta2", C.c_double),
                ("alpha", C.c_double), ("state_degree", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("solves", C.c_int), ("iterations", C.c_int),
                ("refinements", C.c_int), ("fallbacks", C.c_int), ("max_relres", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NewtonOpts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("abs_tol", C.c_double), ("max_iter", C.c_int),
                ("max_backtrack", C.c_int), ("c_armijo", C.c_double), ("max_cg", C.c_int),
                ("gn_iters", C.c_int)]


class NewtonInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("converged", C.c_int),
                ("hessian_applies", C.c_int),
                ("cost", C.c_double * (NEWTON_MAXREC + 1)),
                ("gnorm", C.c_double * (NEWTON_MAXREC + 1)),
                ("cg_iters", C.c_int * NEWTON_MAXREC), ("alpha", C.c_double * NEWTON_MAXREC),
                ("solves", SolveInfo)]

    def as_dict(self):
        it = self.iterations
        return dict(status=self.status, iterations=it, converged=bool(self.converged),
                    hessian_applies=self.hessian_applies,
                    cost=list(self.cost[:it + 1]), gnorm=list(self.gnorm[:it + 1]),
                    cg_iters=list(self.cg_iters[:it]), alpha=list(self.alpha[:it]),
                    solves=self.solves.as_dict())


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    """hinv_allocator: device memory callbacks of a context."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


# Handles still open at interpreter exit are closed by an exit hook, batches
# and networks before problems before contexts, while torch is still whole:
# at module teardown the allocator's free callback would find torch cleared.
_LIVE = {kind: weakref.WeakSet() for kind in ("batch", "cnn", "problem", "ctx")}
_EXIT_HOOK = []


def _close_all():
    for kind in ("batch", "cnn", "problem", "ctx"):
        for obj in list(_LIVE[kind]):
            try:
                obj.close()
            except Exception:
                pass


def _track(kind, obj):
    if not _EXIT_HOOK:
        # registered after torch is imported, so it runs before torch's own hooks
        atexit.register(_close_all)
        _EXIT_HOOK.append(True)
    _LIVE[kind].add(obj)


class TorchAllocator:
    """Device memory for the library's workspaces from PyTorch's caching
    allocator, on the stream the library names (stream-ordered reuse).
    Counts the allocations and frees it serves."""

    def __init__(self, device=0):
        import torch
        self.device = device
        self.allocs = 0
        self.frees = 0
        self.live_bytes = 0

        def alloc(nbytes, stream, _user):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
            except Exception:  # out of memory: the library reports HINV_ENOMEM
                return None
            self.allocs += 1
            self.live_bytes += int(nbytes)
            return p

        def free(ptr, nbytes, _stream, _user):
            torch.cuda.caching_allocator_delete(int(ptr))
            self.frees += 1
            self.live_bytes -= int(nbytes)

        # the callback objects must live as long as the context
        self._alloc, self._free = _ALLOC_FN(alloc), _FREE_FN(free)
        self.struct = Allocator(self._alloc, self._free, None)


EXPORTS = [
    "hinv_ctx_create", "hinv_ctx_destroy", "hinv_ctx_set_stream", "hinv_last_error",
    "hinv_status_string", "hinv_problem_create", "hinv_problem_destroy", "hinv_problem_size",
    "hinv_problem_state_size",
    "hinv_set_data", "hinv_set_solver", "hinv_forward", "hinv_cost", "hinv_observe",
    "hinv_gradient", "hinv_linearize", "hinv_inc_forward", "hinv_inc_adjoint",
    "hinv_hessian_apply", "hinv_prior_apply", "hinv_prior_apply_noalloc", "hinv_prior_solve", "hinv_prior_sample",
    "hinv_map_newton", "hinv_lowrank_eig", "hinv_lowrank_eig_single", "hinv_prior_variance",
    "hinv_posterior_variance", "hinv_posterior_sample", "hinv_posterior_sample_seeded", "hinv_ctx_kernel_timer",
    "hinv_ctx_kernel_timer_read", "hinv_tuner_counts", "hinv_white_noise", "hinv_batch_create", "hinv_batch_destroy",
    "hinv_batch_hessian_apply", "hinv_batch_lowrank_eig", "hinv_state_apply", "hinv_state_solve",
    "hinv_state_solve_fcg", "hinv_cnn_create", "hinv_cnn_destroy", "hinv_cnn_param_count",
    "hinv_cnn_set_params", "hinv_cnn_get_params", "hinv_cnn_forward", "hinv_cnn_gradient",
    "hinv_cnn_train_step", "hinv_cnn_harvest",
]

# timer classes: single-column launches, and the same kernels batched (>= 8 columns)
KCLASS = {"mg_down": 0, "mg_up": 1, "mg_bottom": 2, "pcg_apply": 3, "pcg_update": 4, "gram": 5,
          "mg_down_b": 6, "mg_up_b": 7, "pcg_apply_b": 8, "pcg_update_b": 9}

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Loads libhinv and declares its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libhinv is not built ({path} missing); run "
                           "`python -m paper_1909_03948_amd.build`")
    lib = C.CDLL(path)
    P, I, D, V = C.c_void_p, C.c_int, C.c_double, C.c_void_p
    DP = C.POINTER(C.c_double)
    FP = C.POINTER(C.c_float)
    sig = {
        "hinv_ctx_create": [I, V, C.POINTER(Allocator), C.POINTER(P)],
        "hinv_ctx_destroy": [P],
        "hinv_ctx_set_stream": [P, V],
        "hinv_last_error": [P],
        "hinv_status_string": [I],
        "hinv_problem_create": [P, C.POINTER(ProblemDesc), C.POINTER(P)],
        "hinv_problem_destroy": [P],
        "hinv_problem_size": [P, C.POINTER(I)],
        "hinv_problem_state_size": [P, C.POINTER(I)],
        "hinv_set_data": [P, DP, D],
        "hinv_set_solver": [P, I, D, I],
        "hinv_forward": [P, V, V, C.POINTER(SolveInfo)],
        "hinv_cost": [P, V, V, DP, DP],
        "hinv_observe": [P, V, V],
        "hinv_gradient": [P, V, V, V, V, C.POINTER(SolveInfo)],
        "hinv_linearize": [P, V, V, V],
        "hinv_inc_forward": [P, I, V, I, V, I, C.POINTER(SolveInfo)],
        "hinv_inc_adjoint": [P, I, I, V, I, V, I, V, I, C.POINTER(SolveInfo)],
        "hinv_hessian_apply": [P, I, I, V, I, V, I, C.POINTER(SolveInfo)],
        "hinv_prior_apply": [P, I, V, I, V, I],
        "hinv_prior_apply_noalloc": [P, I, V, I, V, I],
        "hinv_prior_solve": [P, I, V, I, V, I, C.POINTER(SolveInfo)],
        "hinv_prior_sample": [P, I, V, I, V, I, C.POINTER(SolveInfo)],
        "hinv_map_newton": [P, V, V, C.POINTER(NewtonOpts), C.POINTER(NewtonInfo)],
        "hinv_lowrank_eig": [P, I, I, I, V, I, I, DP, V, I, C.POINTER(SolveInfo)],
        "hinv_posterior_sample": [P, V, I, DP, V, I, I, V, I, V, I, C.POINTER(SolveInfo)],
        "hinv_lowrank_eig_single": [P, I, I, V, I, I, DP, V, I, C.POINTER(SolveInfo)],
        "hinv_posterior_sample_seeded": [P, V, I, DP, V, I, C.c_uint64, C.c_uint64, C.c_int64, I, V, I,
                                         C.POINTER(SolveInfo)],
        "hinv_prior_variance": [P, I, V, I, V, DP, C.POINTER(SolveInfo)],
        "hinv_posterior_variance": [P, V, I, DP, V, I, V],
        "hinv_ctx_kernel_timer": [P, I, I, I],
        "hinv_white_noise": [P, C.c_uint64, C.c_uint64, C.c_int64, I, V, I],
        "hinv_tuner_counts": [C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)],
        "hinv_ctx_kernel_timer_read": [P, I, C.POINTER(I), C.POINTER(C.c_long), DP, DP],
        "hinv_batch_create": [P, I, C.POINTER(P), C.POINTER(P)],
        "hinv_batch_destroy": [P],
        "hinv_batch_hessian_apply": [P, I, I, C.POINTER(V), C.POINTER(V), C.POINTER(SolveInfo)],
        "hinv_batch_lowrank_eig": [P, I, I, I, C.POINTER(V), I, DP, C.POINTER(V),
                                   C.POINTER(SolveInfo)],
        "hinv_state_apply": [P, I, V, I, V, I],
        "hinv_state_solve": [P, I, V, I, V, I, C.POINTER(SolveInfo)],
        "hinv_state_solve_fcg": [P, P, V, V, D, I, I, C.POINTER(FcgInfo)],
        "hinv_cnn_create": [P, C.POINTER(P)],
        "hinv_cnn_destroy": [P],
        "hinv_cnn_param_count": [],
        "hinv_cnn_set_params": [P, FP, I],
        "hinv_cnn_get_params": [P, FP, I],
        "hinv_cnn_forward": [P, I, I, V, V],
        "hinv_cnn_gradient": [P, I, I, V, V, I, DP, FP],
        "hinv_cnn_train_step": [P, I, I, V, V, I, C.c_float, DP],
        "hinv_cnn_harvest": [P, I, C.c_uint64, I, V, V, C.POINTER(SolveInfo)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_char_p if name in ("hinv_last_error", "hinv_status_string") else C.c_int
    _lib = lib
    return lib


def tuner_counts():
    """(launch shapes timed, launch shapes taken from the HINV_TUNE_CACHE file) in this process."""
    lib = load()
    t, c = C.c_longlong(), C.c_longlong()
    lib.hinv_tuner_counts(C.byref(t), C.byref(c))
    return t.value, c.value


class HinvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def _ptr(t):
    """Device pointer of a CUDA float64 tensor whose last dimension is contiguous."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("expected a CUDA float64 tensor")
    if t.dim() > 0 and t.numel() > 0 and t.stride(-1) != 1:
        raise ValueError("last dimension must be contiguous")
    return C.c_void_p(t.data_ptr())


def _same(*counts):
    """Every multivector of a call has the same number of columns."""
    if len(set(counts)) != 1:
        raise ValueError(f"column counts differ: {counts}")


def _vec(t, n):
    """Pointer of a vector of at least n entries (a 1-D tensor or one packed row)."""
    if t.dim() != 1 and not (t.dim() == 2 and t.shape[0] == 1):
        raise ValueError("expected a vector")
    if t.numel() < n:
        raise ValueError(f"vector has {t.numel()} entries, needs {n}")
    return _ptr(t)


def _cols(t, n):
    """(pointer, ncols, ld) of a multivector given as a (c, ld) or (n,) tensor."""
    if t.numel() == 0:
        return _ptr(t), 0, n
    if t.dim() == 1:
        if t.shape[0] < n:
            raise ValueError("vector too short")
        return _ptr(t), 1, max(n, t.shape[0])
    if t.shape[1] < n:
        raise ValueError("multivector rows shorter than n")
    return _ptr(t), t.shape[0], t.stride(0)


class Context:
    """hinv_ctx on a device and stream (default: torch's current stream).
    allocator: "torch" (default: workspaces come from PyTorch's caching
    allocator), a TorchAllocator, or None (the library's hipMalloc)."""

    def __init__(self, device: int = 0, stream=None, allocator="torch"):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        if allocator == "torch":
            allocator = TorchAllocator(device)
        self.allocator = allocator
        h = C.c_void_p()
        ap = C.byref(allocator.struct) if allocator is not None else None
        rc = self.lib.hinv_ctx_create(device, C.c_void_p(stream), ap, C.byref(h))
        if rc != HINV_OK:
            raise HinvError(rc, self.lib.hinv_last_error(None).decode())
        self.h = h
        _track("ctx", self)

    def close(self):
        if getattr(self, "h", None):
            self.lib.hinv_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self):
        return self.lib.hinv_last_error(self.h).decode()

    def kernel_timer(self, name, enable=True, period=16):
        rc = self.lib.hinv_ctx_kernel_timer(self.h, KCLASS[name], int(enable), period)
        if rc != HINV_OK:
            raise HinvError(rc, self.error())

    def kernel_timer_read(self, name):
        """dict(timed, launches, ms, work) of the sampled launches of a class."""
        t, n, ms, w = C.c_int(), C.c_long(), C.c_double(), C.c_double()
        rc = self.lib.hinv_ctx_kernel_timer_read(self.h, KCLASS[name], C.byref(t), C.byref(n),
                                                 C.byref(ms), C.byref(w))
        if rc != HINV_OK:
            raise HinvError(rc, self.error())
        return dict(timed=t.value, launches=n.value, ms=ms.value, work=w.value)


class Problem:
    """Binding of hinv_problem; method names follow the C functions."""

    def __init__(self, ctx: Context, N, gamma, delta, obs_xy=None, d_obs=None, sigma=0.01,
                 m_prior=-2.0, beta=float("nan"), precision=PREC_FP64, rtol=1e-10, max_iter=0,
                 theta=None, state_degree=1):
        """theta: None (Theta = I) or (theta1, theta2, alpha) of the prior's anisotropic tensor.
        state_degree: 1 (P1 state) or 2 (P2 state: state vectors have ns = (2N+1)^2 entries)."""
        self.ctx, self.lib = ctx, ctx.lib
        xy = np.ascontiguousarray(np.zeros((0, 2)) if obs_xy is None else obs_xy, dtype=np.float64)
        q = xy.shape[0]
        self._xy = xy.reshape(-1)
        self._d = None if d_obs is None else np.ascontiguousarray(d_obs, dtype=np.float64)
        DP = C.POINTER(C.c_double)
        desc = ProblemDesc(N=N, gamma=gamma, delta=delta, beta=beta, m_prior=m_prior, q=q,
                           obs_xy=self._xy.ctypes.data_as(DP) if q else None,
                           d_obs=self._d.ctypes.data_as(DP) if self._d is not None else None,
                           sigma=sigma, precision=precision, rtol=rtol, max_iter=max_iter,
                           theta1=theta[0] if theta else 0.0, theta2=theta[1] if theta else 0.0,
                           alpha=theta[2] if theta else 0.0, state_degree=state_degree)
        h = C.c_void_p()
        self._check(self.lib.hinv_problem_create(ctx.h, C.byref(desc), C.byref(h)), allow=())
        self.h = h
        _track("problem", self)
        self.N, self.n, self.q = N, (N + 1) ** 2, q
        nsv = C.c_int()
        self._check(self.lib.hinv_problem_state_size(self.h, C.byref(nsv)), allow=())
        self.ns = nsv.value

    def _check(self, rc, allow=(HINV_ENOCONV,)):
        if rc != HINV_OK and rc not in allow:
            raise HinvError(rc, self.ctx.error() or self.lib.hinv_status_string(rc).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.hinv_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_data(self, d_obs=None, sigma=float("nan")):
        DP = C.POINTER(C.c_double)
        self._d = None if d_obs is None else np.ascontiguousarray(d_obs, dtype=np.float64)
        p = self._d.ctypes.data_as(DP) if self._d is not None else None
        self._check(self.lib.hinv_set_data(self.h, p, sigma), allow=())

    def set_solver(self, precision, rtol, max_iter=0):
        self._check(self.lib.hinv_set_solver(self.h, precision, rtol, max_iter), allow=())

    def forward(self, m, u):
        info = SolveInfo()
        rc = self._check(self.lib.hinv_forward(self.h, _vec(m, self.n), _vec(u, self.ns), C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def cost(self, m, u):
        mis, reg = C.c_double(), C.c_double()
        self._check(self.lib.hinv_cost(self.h, _vec(m, self.n), _vec(u, self.ns), C.byref(mis), C.byref(reg)),
                    allow=())
        return mis.value, reg.value

    def observe(self, u, Bu):
        self._check(self.lib.hinv_observe(self.h, _vec(u, self.ns), _vec(Bu, self.q)), allow=())

    def gradient(self, m, u, p, g):
        info = SolveInfo()
        rc = self._check(self.lib.hinv_gradient(self.h, _vec(m, self.n), _vec(u, self.ns), _vec(p, self.ns),
                                                _vec(g, self.n), C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def linearize(self, m, u, p):
        self._check(self.lib.hinv_linearize(self.h, _vec(m, self.n), _vec(u, self.ns), _vec(p, self.ns)),
                    allow=())

    def inc_forward(self, mhat, uhat):
        pm, nc, ldm = _cols(mhat, self.n)
        pu, nc2, ldu = _cols(uhat, self.ns)
        _same(nc, nc2)
        info = SolveInfo()
        rc = self._check(self.lib.hinv_inc_forward(self.h, nc, pm, ldm, pu, ldu, C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def inc_adjoint(self, mhat, uhat, phat, gauss_newton=False):
        pm, nc, ldm = _cols(mhat, self.n)
        pu, nc2, ldu = _cols(uhat, self.ns)
        pp, nc3, ldp = _cols(phat, self.ns)
        _same(nc, nc2, nc3)
        info = SolveInfo()
        rc = self._check(self.lib.hinv_inc_adjoint(self.h, nc, int(gauss_newton), pm, ldm, pu, ldu,
                                                   pp, ldp, C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def hessian_apply(self, mode, mhat, out):
        pm, nc, ldm = _cols(mhat, self.n)
        po, nc2, ldo = _cols(out, self.n)
        _same(nc, nc2)
        info = SolveInfo()
        rc = self._check(self.lib.hinv_hessian_apply(self.h, mode, nc, pm, ldm, po, ldo, C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def prior_apply(self, x, y):
        px, nc, ldx = _cols(x, self.n)
        py, nc2, ldy = _cols(y, self.n)
        _same(nc, nc2)
        self._check(self.lib.hinv_prior_apply(self.h, nc, px, ldx, py, ldy), allow=())

    def prior_apply_noalloc(self, x, y):
        """y = R x through the entry point that allocates nothing."""
        px, nc, ldx = _cols(x, self.n)
        py, nc2, ldy = _cols(y, self.n)
        _same(nc, nc2)
        self._check(self.lib.hinv_prior_apply_noalloc(self.h, nc, px, ldx, py, ldy), allow=())

    def prior_solve(self, x, y):
        px, nc, ldx = _cols(x, self.n)
        py, nc2, ldy = _cols(y, self.n)
        _same(nc, nc2)
        info = SolveInfo()
        rc = self._check(self.lib.hinv_prior_solve(self.h, nc, px, ldx, py, ldy, C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def prior_sample(self, eta, out):
        pe, ns, lde = _cols(eta, 6 * self.N * self.N)
        po, ns2, ldo = _cols(out, self.n)
        _same(ns, ns2)
        info = SolveInfo()
        rc = self._check(self.lib.hinv_prior_sample(self.h, ns, pe, lde, po, ldo, C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def white_noise(self, seed, stream, first, eta):
        pe, ns, lde = _cols(eta, 6 * self.N * self.N)
        self._check(self.lib.hinv_white_noise(self.h, seed, stream, first, ns, pe, lde), allow=())

    def map_newton(self, m_map, m0=None, rel_tol=1e-6, abs_tol=0.0, max_iter=50, max_backtrack=10,
                   c_armijo=1e-4, max_cg=500, gn_iters=5):
        opts = NewtonOpts(rel_tol=rel_tol, abs_tol=abs_tol, max_iter=max_iter,
                          max_backtrack=max_backtrack, c_armijo=c_armijo, max_cg=max_cg,
                          gn_iters=int(gn_iters))
        info = NewtonInfo()
        rc = self.lib.hinv_map_newton(self.h, None if m0 is None else _vec(m0, self.n), _vec(m_map, self.n),
                                      C.byref(opts), C.byref(info))
        self._check(rc, allow=(HINV_ENOCONV, HINV_ESTATE))
        return info.as_dict() | {"rc": rc}

    def state_apply(self, x, y):
        px, nc, ldx = _cols(x, self.ns)
        py, nc2, ldy = _cols(y, self.ns)
        _same(nc, nc2)
        self._check(self.lib.hinv_state_apply(self.h, nc, px, ldx, py, ldy), allow=())

    def state_solve(self, b, x):
        pb, nc, ldb = _cols(b, self.ns)
        px, nc2, ldx = _cols(x, self.ns)
        _same(nc, nc2)
        info = SolveInfo()
        rc = self._check(self.lib.hinv_state_solve(self.h, nc, pb, ldb, px, ldx, C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def state_solve_fcg(self, b, x, net=None, rtol=1e-10, max_iter=200, truncation=1):
        info = FcgInfo()
        rc = self._check(self.lib.hinv_state_solve_fcg(self.h, None if net is None else net.h, _vec(b, self.n),
                                                       _vec(x, self.n),
                                                       rtol, max_iter, truncation, C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def cnn_harvest(self, npairs, seed, crop, inp, target):
        """inp: CUDA float32 (npairs, 3, crop, crop); target: (npairs, 4, crop, crop)."""
        _fcheck(inp, (npairs, 3, crop, crop))
        _fcheck(target, (npairs, 4, crop, crop))
        info = SolveInfo()
        rc = self._check(self.lib.hinv_cnn_harvest(self.h, npairs, seed, crop, C.c_void_p(inp.data_ptr()),
                                                   C.c_void_p(target.data_ptr()), C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def lowrank_eig(self, omega, k, V, mode=HESS_MISFIT, tprod=TPROD_FP64):
        po, s, ldo = _cols(omega, self.n)
        pv, kv, ldv = _cols(V, self.n)
        if not 1 <= k <= min(s, kv):
            raise ValueError("need 1 <= k <= number of probe vectors and of V's columns")
        lam = (C.c_double * k)()
        info = SolveInfo()
        rc = self._check(self.lib.hinv_lowrank_eig(self.h, mode, tprod, s, po, ldo, k, lam, pv, ldv,
                                                   C.byref(info)))
        return np.array(lam[:]), info.as_dict() | {"rc": rc}

    def lowrank_eig_single(self, omega, k, V, mode=HESS_MISFIT):
        """Single-pass eigensolver (Alg. 3): (lambda[k], info); V (>= k, n) receives V_k."""
        po, s, ldo = _cols(omega, self.n)
        pv, kv, ldv = _cols(V, self.n)
        if not 1 <= k <= min(s, kv):
            raise ValueError("need 1 <= k <= number of probe vectors and of V's columns")
        lam = (C.c_double * k)()
        info = SolveInfo()
        rc = self._check(self.lib.hinv_lowrank_eig_single(self.h, mode, s, po, ldo, k, lam, pv, ldv,
                                                          C.byref(info)))
        return np.array(lam[:]), info.as_dict() | {"rc": rc}

    def prior_variance(self, omega, diag):
        """diag(R^-1) by Eq. eq:prior_mvar with the s columns of omega: (mu[s], info)."""
        po, s, ldo = _cols(omega, self.n)
        _vec(diag, self.n)
        mu = (C.c_double * max(s, 1))()
        info = SolveInfo()
        rc = self._check(self.lib.hinv_prior_variance(self.h, s, po, ldo, _ptr(diag), mu, C.byref(info)))
        return np.array(mu[:s]), info.as_dict() | {"rc": rc}

    def posterior_variance(self, prior_diag, lam, V, diag):
        """diag = prior_diag - sum lambda/(1+lambda) v^2 (Eq. eq:post_mvar)."""
        k = len(lam)
        _vec(prior_diag, self.n)
        _vec(diag, self.n)
        pv, kv, ldv = _cols(V, self.n)
        if kv < k:
            raise ValueError("V has fewer columns than eigenvalues")
        lam_arr = (C.c_double * max(k, 1))(*[float(x) for x in lam])
        self._check(self.lib.hinv_posterior_variance(self.h, _ptr(prior_diag), k, lam_arr, pv, ldv,
                                                     _ptr(diag)), allow=())

    def posterior_sample_seeded(self, m_map, lam, V, seed, stream, first, out):
        """out[j] = posterior sample first + j of the counter-based stream (seed, stream)."""
        k = len(lam)
        lam_arr = (C.c_double * max(k, 1))(*[float(x) for x in lam])
        pv, kv, ldv = _cols(V, self.n)
        if kv < k:
            raise ValueError("V has fewer columns than eigenvalues")
        po, ns, ldo = _cols(out, self.n)
        info = SolveInfo()
        rc = self._check(self.lib.hinv_posterior_sample_seeded(self.h, _vec(m_map, self.n), k, lam_arr, pv, ldv,
                                                               seed, stream, first, ns, po, ldo, C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def posterior_sample(self, m_map, lam, V, eta, out):
        k = len(lam)
        lam_arr = (C.c_double * max(k, 1))(*[float(x) for x in lam])
        pv, kv, ldv = _cols(V, self.n)
        if kv < k:
            raise ValueError("V has fewer columns than eigenvalues")
        pe, ns, lde = _cols(eta, 6 * self.N * self.N)
        po, ns2, ldo = _cols(out, self.n)
        _same(ns, ns2)
        info = SolveInfo()
        rc = self._check(self.lib.hinv_posterior_sample(self.h, _vec(m_map, self.n), k, lam_arr, pv, ldv, ns,
                                                        pe, lde, po, ldo, C.byref(info)))
        return info.as_dict() | {"rc": rc}


def _fcheck(t, shape):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError("expected a CUDA float32 tensor")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"expected a contiguous tensor of shape {shape}")


class Cnn:
    """Binding of hinv_cnn (the residual CNN of the learned correction).
    Images: CUDA float32 tensors, input (B, 3, S, S), output / target (B, S, S)."""

    def __init__(self, ctx: Context):
        self.ctx, self.lib = ctx, ctx.lib
        h = C.c_void_p()
        rc = self.lib.hinv_cnn_create(ctx.h, C.byref(h))
        if rc != HINV_OK:
            raise HinvError(rc, ctx.error() or self.lib.hinv_status_string(rc).decode())
        self.h = h
        _track("cnn", self)
        self.nparams = self.lib.hinv_cnn_param_count()

    def _check(self, rc):
        if rc != HINV_OK:
            raise HinvError(rc, self.ctx.error() or self.lib.hinv_status_string(rc).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.hinv_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        if a.size != self.nparams:
            raise ValueError("parameter count mismatch")
        self._check(self.lib.hinv_cnn_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))

    # (c_out, c_in) of the six convolutions: 3 -> 32, four 32 -> 32, 32 -> 1
    LAYERS = ((32, 3), (32, 32), (32, 32), (32, 32), (32, 32), (1, 32))

    def he_init(self, seed=0):
        """Seeded He-normal weights (std sqrt(2 / (9 c_in)), the last layer's
        scaled by 0.1 so the initial correction is small), zero biases, packed
        per layer as W[c_out][c_in][3][3] then b[c_out]; resets Adam."""
        rng = np.random.default_rng(seed)
        parts = []
        for li, (co, ci) in enumerate(self.LAYERS):
            std = np.sqrt(2.0 / (9.0 * ci)) * (0.1 if li == len(self.LAYERS) - 1 else 1.0)
            parts += [std * rng.standard_normal(co * ci * 9), np.zeros(co)]
        self.set_params(np.concatenate(parts))

    def get_params(self):
        a = np.zeros(self.nparams, dtype=np.float32)
        self._check(self.lib.hinv_cnn_get_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    def forward(self, inp, out):
        B, S = inp.shape[0], inp.shape[-1]
        _fcheck(inp, (B, 3, S, S))
        _fcheck(out, (B, S, S))
        self._check(self.lib.hinv_cnn_forward(self.h, B, S, C.c_void_p(inp.data_ptr()), C.c_void_p(out.data_ptr())))

    @staticmethod
    def _tchan(target, B, S):
        if target.dim() == 3:
            _fcheck(target, (B, S, S))
            return 1
        _fcheck(target, (B, 4, S, S))
        return 4

    def gradient(self, inp, target):
        """target (B, S, S): relative L2 loss; (B, 4, S, S) = (t, wE, wN, diag):
        relative energy norm."""
        B, S = inp.shape[0], inp.shape[-1]
        _fcheck(inp, (B, 3, S, S))
        tc = self._tchan(target, B, S)
        g = np.zeros(self.nparams, dtype=np.float32)
        L = C.c_double()
        self._check(self.lib.hinv_cnn_gradient(self.h, B, S, C.c_void_p(inp.data_ptr()),
                                               C.c_void_p(target.data_ptr()), tc, C.byref(L),
                                               g.ctypes.data_as(C.POINTER(C.c_float))))
        return L.value, g

    def train_step(self, inp, target, lr):
        B, S = inp.shape[0], inp.shape[-1]
        _fcheck(inp, (B, 3, S, S))
        tc = self._tchan(target, B, S)
        L = C.c_double()
        self._check(self.lib.hinv_cnn_train_step(self.h, B, S, C.c_void_p(inp.data_ptr()),
                                                 C.c_void_p(target.data_ptr()), tc, float(lr), C.byref(L)))
        return L.value


class Batch:
    """Binding of hinv_batch: independent problems advanced together.  Vectors
    are given per problem as (c, n_i) CUDA float64 tensors (row = column of the
    C multivector, rows contiguous and packed)."""

    def __init__(self, ctx: Context, problems):
        self.ctx, self.lib = ctx, ctx.lib
        self.problems = list(problems)  # keeps the problems alive
        arr = (C.c_void_p * len(self.problems))(*[p.h.value for p in self.problems])
        h = C.c_void_p()
        rc = self.lib.hinv_batch_create(ctx.h, len(self.problems), arr, C.byref(h))
        if rc != HINV_OK:
            raise HinvError(rc, ctx.error() or self.lib.hinv_status_string(rc).decode())
        self.h = h
        _track("batch", self)

    def _check(self, rc, allow=(HINV_ENOCONV,)):
        if rc != HINV_OK and rc not in allow:
            raise HinvError(rc, self.ctx.error() or self.lib.hinv_status_string(rc).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.hinv_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, ts, ncol):
        if len(ts) != len(self.problems):
            raise ValueError("one tensor per problem")
        out = []
        for t, p in zip(ts, self.problems):
            if t.dim() != 2 or t.shape[0] < ncol or t.shape[1] != p.n or (t.numel() and t.stride(0) != p.n):
                raise ValueError("expected a packed (c, n_i) tensor per problem")
            out.append(_ptr(t).value)
        return (C.c_void_p * len(out))(*out)

    def hessian_apply(self, mode, mhats, outs):
        nrhs = mhats[0].shape[0]
        info = SolveInfo()
        rc = self._check(self.lib.hinv_batch_hessian_apply(self.h, mode, nrhs, self._ptrs(mhats, nrhs),
                                                           self._ptrs(outs, nrhs), C.byref(info)))
        return info.as_dict() | {"rc": rc}

    def lowrank_eig(self, omegas, k, Vs, mode=HESS_MISFIT, tprod=TPROD_FP64):
        s = omegas[0].shape[0]
        lam = (C.c_double * (k * len(self.problems)))()
        info = SolveInfo()
        rc = self._check(self.lib.hinv_batch_lowrank_eig(self.h, mode, tprod, s, self._ptrs(omegas, s), k,
                                                         lam, self._ptrs(Vs, k), C.byref(info)))
        return np.array(lam[:]).reshape(len(self.problems), k), info.as_dict() | {"rc": rc}

