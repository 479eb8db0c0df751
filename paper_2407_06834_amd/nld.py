"""Thin ctypes binding of libnld (C ABI in include/nld.h).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  PyTorch supplies device memory
and the current stream.

The functions mirror the C entry points (nfft_plan, nfft_plan_destroy, degree_vector,
anova_matvec, laplacian_matvec, pcg_solve, features_from_image); ``Plan`` wraps a plan
handle for convenience.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnld.so")

NLD_OK, NLD_E_INVAL, NLD_E_NOMEM, NLD_E_HIP, NLD_E_NOCONV, NLD_E_BREAKDOWN, NLD_E_STATE = range(7)
NLD_FP32, NLD_FP64 = 0, 1
STATUS_NAMES = {0: "OK", 1: "E_INVAL", 2: "E_NOMEM", 3: "E_HIP", 4: "E_NOCONV", 5: "E_BREAKDOWN",
                6: "E_STATE"}

# Entry points declared in include/nld.h
SYMBOLS = ("nfft_plan", "nfft_plan_update_kernel", "nfft_plan_destroy", "nfft_plan_window_info", "nfft_plan_size",
           "degree_vector", "anova_matvec", "laplacian_matvec", "pcg_solve", "pcg_solve_batched", "adjoint_solve",
           "features_from_image", "mis_scores", "mis_scores_noalloc", "nld_last_error")


class KernelDesc(ctypes.Structure):
    _fields_ = [("n_windows", ctypes.c_int32), ("win_dim", ctypes.POINTER(ctypes.c_int32)),
                ("win_feat", ctypes.POINTER(ctypes.c_int32)),
                ("sigma", ctypes.POINTER(ctypes.c_double)),
                ("weight", ctypes.POINTER(ctypes.c_double)), ("bandwidth", ctypes.c_int32),
                ("win_bandwidth", ctypes.POINTER(ctypes.c_int32)), ("cutoff", ctypes.c_int32),
                ("oversampling", ctypes.c_double), ("matvec_tol", ctypes.c_double),
                ("prec", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("max_grid", ctypes.c_int32)]


class WindowInfo(ctypes.Structure):
    _fields_ = [("dims_kept", ctypes.c_int32), ("bandwidth", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("cutoff", ctypes.c_int32),
                ("compression", ctypes.c_double * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3)]


class PcgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("use_u0", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("deflate", ctypes.c_int32),
                ("true_residual", ctypes.c_int32), ("timing", ctypes.c_int32)]


class PcgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("relres_rec", ctypes.c_double),
                ("relres_true", ctypes.c_double), ("kappa_est", ctypes.c_double),
                ("ms_solve", ctypes.c_double), ("ms_matvec", ctypes.c_double),
                ("matvecs_timed", ctypes.c_int32), ("status", ctypes.c_int32),
                ("u0_rejected", ctypes.c_int32)]

    def as_dict(self):
        return {"iters": self.iters, "relres_rec": self.relres_rec,
                "relres_true": self.relres_true, "kappa_est": self.kappa_est,
                "ms_solve": self.ms_solve, "ms_matvec": self.ms_matvec,
                "matvecs_timed": self.matvecs_timed,
                "status": STATUS_NAMES.get(self.status, self.status),
                "u0_rejected": bool(self.u0_rejected)}


_lib = None


def load() -> ctypes.CDLL:
    """Load libnld.so from the package directory; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libnld.so not found at {LIB_PATH}; run "
                          "`python -m paper_2407_06834_amd.build` (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "nfft_plan": [ctypes.POINTER(P), P, I64, I32, ctypes.POINTER(KernelDesc), P],
        "nfft_plan_destroy": [P],
        "nfft_plan_update_kernel": [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), P],
        "nfft_plan_window_info": [P, I32, ctypes.POINTER(WindowInfo)],
        "nfft_plan_size": [P, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(I32)],
        "degree_vector": [P, P, P],
        "anova_matvec": [P, P, P, P],
        "laplacian_matvec": [P, P, P, P],
        "pcg_solve": [P, D, P, P, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgInfo), P],
        "pcg_solve_batched": [ctypes.POINTER(P), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(P),
                              ctypes.POINTER(P), I32, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgInfo), P],
        "adjoint_solve": [P, D, P, P, P, P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(PcgOpts),
                          ctypes.POINTER(PcgInfo), P],
        "features_from_image": [P, I32, I32, I32, I32, I32, P, P],
        "mis_scores": [P, I64, I32, P, I32, I32, P, P],
        "mis_scores_noalloc": [P, I64, I32, P, I32, I32, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.nld_last_error.argtypes = []
    lib.nld_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


class NldError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status: int):
    if status != NLD_OK:
        raise NldError(status, load().nld_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype(prec: int):
    return torch.float32 if prec == NLD_FP32 else torch.float64


def _precond(p) -> int:
    """Preconditioner code: False/'none' 0, True/'jacobi' 1 (P_a), 'l2' 2 (P_b')."""
    if isinstance(p, str):
        return {"none": 0, "jacobi": 1, "l2": 2}[p]
    return int(p)


def _vec(t: torch.Tensor, n: int, dtype, name: str):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() == n):
        raise ValueError(f"{name}: expected a contiguous {dtype} CUDA tensor with {n} elements")
    return ctypes.c_void_p(t.data_ptr())


def features_from_image(img: torch.Tensor, rho: int, with_pos: bool = True, stream=None):
    """SoA features (d, N) of a 2-D image tensor (float32 or float64, on the GPU)."""
    if img.dim() != 2 or not img.is_cuda or img.dtype not in (torch.float32, torch.float64):
        raise ValueError("img: expected a 2-D float32/float64 CUDA tensor")
    img = img.contiguous()
    n1, n2 = img.shape
    prec = NLD_FP32 if img.dtype == torch.float32 else NLD_FP64
    d = (2 if with_pos else 0) + (2 * rho + 1) ** 2
    F = torch.empty((d, n1 * n2), dtype=img.dtype, device=img.device)
    _check(load().features_from_image(ctypes.c_void_p(img.data_ptr()), n1, n2, rho,
                                      1 if with_pos else 0, prec, ctypes.c_void_p(F.data_ptr()),
                                      _stream(stream)))
    return F


@dataclass
class WindowParams:
    dims_kept: int
    bandwidth: int
    grid: int
    cutoff: int
    compression: tuple
    lo: tuple
    hi: tuple


class Plan:
    """A plan of the fast ANOVA summation over fixed features (see nfft_plan in nld.h)."""

    def __init__(self, features: torch.Tensor, windows, sigma, weight, bandwidth: int = 0,
                 cutoff: int = 0, oversampling: float = 2.0, matvec_tol: float = 1e-6,
                 win_bandwidth=None, tile: int = 0, max_grid: int = 0, stream=None):
        lib = load()
        if features.dim() != 2 or not features.is_cuda:
            raise ValueError("features: expected a (d, N) CUDA tensor")
        if features.dtype not in (torch.float32, torch.float64):
            raise ValueError("features: float32 or float64")
        self.features = features.contiguous()   # kept alive with the plan
        self.prec = NLD_FP32 if features.dtype == torch.float32 else NLD_FP64
        self.dtype = features.dtype
        self.d, self.N = self.features.shape
        L = len(windows)
        self.L = L
        self._wd = (ctypes.c_int32 * L)(*[len(w) for w in windows])
        flat = [int(c) for w in windows for c in w]
        self._wf = (ctypes.c_int32 * max(1, len(flat)))(*flat)
        self._sig = (ctypes.c_double * L)(*[float(s) for s in sigma])
        self._wt = (ctypes.c_double * L)(*[float(w) for w in weight])
        self._wbw = (ctypes.c_int32 * L)(*win_bandwidth) if win_bandwidth is not None else None
        desc = KernelDesc(L, self._wd, self._wf, self._sig, self._wt, int(bandwidth),
                          self._wbw if self._wbw is not None else None, int(cutoff),
                          float(oversampling), float(matvec_tol), self.prec, int(tile),
                          int(max_grid))
        h = ctypes.c_void_p()
        _check(lib.nfft_plan(ctypes.byref(h), ctypes.c_void_p(self.features.data_ptr()), self.N,
                             self.d, ctypes.byref(desc), _stream(stream)))
        self.handle = h

    def update_kernel(self, sigma, weight, stream=None) -> bool:
        """New (sigma_l, w_l) on the same nodes (see nfft_plan_update_kernel in nld.h).
        Returns False, leaving the plan unchanged, when the widths need a new plan."""
        sig = (ctypes.c_double * self.L)(*[float(x) for x in sigma])
        wt = (ctypes.c_double * self.L)(*[float(x) for x in weight])
        st = load().nfft_plan_update_kernel(self.handle, sig, wt, _stream(stream))
        if st == NLD_E_STATE:
            return False
        _check(st)
        self._sig, self._wt = sig, wt
        return True

    def close(self):
        if getattr(self, "handle", None):
            _check(load().nfft_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def window_info(self, l: int) -> WindowParams:
        info = WindowInfo()
        _check(load().nfft_plan_window_info(self.handle, l, ctypes.byref(info)))
        t = info.dims_kept
        return WindowParams(t, info.bandwidth, info.grid, info.cutoff,
                            tuple(info.compression[:t]), tuple(info.lo[:t]), tuple(info.hi[:t]))

    def degree_vector(self, stream=None) -> torch.Tensor:
        D = torch.empty(self.N, dtype=torch.float64, device=self.features.device)
        _check(load().degree_vector(self.handle, ctypes.c_void_p(D.data_ptr()), _stream(stream)))
        return D

    def anova_matvec(self, v: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        out = torch.empty_like(v) if out is None else out
        _check(load().anova_matvec(self.handle, _vec(v, self.N, self.dtype, "v"),
                                   _vec(out, self.N, self.dtype, "out"), _stream(stream)))
        return out

    def laplacian_matvec(self, v: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        out = torch.empty_like(v) if out is None else out
        _check(load().laplacian_matvec(self.handle, _vec(v, self.N, self.dtype, "v"),
                                       _vec(out, self.N, self.dtype, "out"), _stream(stream)))
        return out

    def pcg_solve(self, alpha: float, f: torch.Tensor, u0: torch.Tensor | None = None,
                  tol: float = 1e-6, maxit: int = 500, precond: bool = True,
                  deflate: bool = True, true_residual: bool = False, out=None, stream=None,
                  raise_on_noconv: bool = False, timing: bool = False,
                  u0_guard: str = "finite"):
        """Solve (I + alpha L~) u = f.  Returns (u, info dict).  With a warm start u0,
        u0_guard "finite" falls back to u0 = f when u0's initial residual is not finite,
        "residual" also when it exceeds the residual of u0 = f (one more product), "scaled"
        starts from the energy-optimal multiple of u0 - mean(u0) (see use_u0 in nld.h)."""
        u = torch.empty_like(f) if out is None else out
        if u0 is not None:
            u.copy_(u0)
        mode = 0 if u0 is None else {"finite": 1, "residual": 2, "scaled": 3}[u0_guard]
        opts = PcgOpts(float(tol), int(maxit), mode, _precond(precond),
                       int(bool(deflate)), int(bool(true_residual)), int(bool(timing)))
        info = PcgInfo()
        st = load().pcg_solve(self.handle, float(alpha), _vec(f, self.N, self.dtype, "f"),
                              _vec(u, self.N, self.dtype, "u"), ctypes.byref(opts),
                              ctypes.byref(info), _stream(stream))
        if st not in (NLD_OK, NLD_E_NOCONV, NLD_E_BREAKDOWN) or (raise_on_noconv and st != NLD_OK):
            _check(st)
        return u, info.as_dict()


    def adjoint_solve(self, alpha: float, f: torch.Tensor, u: torch.Tensor, g: torch.Tensor,
                      tol: float = 1e-10, maxit: int = 500, stream=None):
        """Adjoint solve A p = g and the gradient (see adjoint_solve in nld.h).
        Returns (p, grad, info) with grad = [dJ/dlog alpha, dJ/dlog sigma_l..., dJ/dw_l...]."""
        import numpy as np
        p = torch.empty_like(g)
        grad = (ctypes.c_double * (1 + 2 * self.L))()
        opts = PcgOpts(float(tol), int(maxit), 0, 1, 1, 0, 0)
        info = PcgInfo()
        st = load().adjoint_solve(self.handle, float(alpha), _vec(f, self.N, self.dtype, "f"),
                                  _vec(u, self.N, self.dtype, "u"), _vec(g, self.N, self.dtype, "g"),
                                  _vec(p, self.N, self.dtype, "p"), grad, ctypes.byref(opts),
                                  ctypes.byref(info), _stream(stream))
        if st not in (NLD_OK, NLD_E_NOCONV):
            _check(st)
        return p, np.array(grad[:], dtype=np.float64), info.as_dict()


def nfft_plan(features, windows, sigma, weight, **kw) -> Plan:
    return Plan(features, windows, sigma, weight, **kw)


def nfft_plan_update_kernel(plan: Plan, sigma, weight, **kw) -> bool:
    return plan.update_kernel(sigma, weight, **kw)


def nfft_plan_destroy(plan: Plan):
    plan.close()


def degree_vector(plan: Plan, **kw):
    return plan.degree_vector(**kw)


def anova_matvec(plan: Plan, v, out=None, **kw):
    return plan.anova_matvec(v, out=out, **kw)


def laplacian_matvec(plan: Plan, v, out=None, **kw):
    return plan.laplacian_matvec(v, out=out, **kw)


def pcg_solve(plan: Plan, alpha, f, **kw):
    return plan.pcg_solve(alpha, f, **kw)


def window_table(rho: int, with_pos: bool = True):
    """Fixed window grouping of the feature rows (position + centre first, then the other
    patch offsets in raster order in chunks of three)."""
    P = 2 * rho + 1
    base = 2 if with_pos else 0
    centre = base + rho * P + rho
    rest = [base + p for p in range(P * P) if not (with_pos and base + p == centre)]
    wins = [[0, 1, centre]] if with_pos else []
    wins += [rest[s:s + 3] for s in range(0, len(rest), 3)]
    return wins


def mis_scores(features: torch.Tensor, target: torch.Tensor, bins: int = 0, stream=None,
               out=None, noalloc: bool = False):
    """Mutual information score (float64, on the GPU) of every feature row of the SoA matrix
    (d, N) against the target (N); see mis_scores in nld.h.  noalloc=True calls
    mis_scores_noalloc (the library allocates nothing; pass `out` to allocate nothing here
    either)."""
    if features.dim() != 2 or not features.is_cuda:
        raise ValueError("features: expected a 2-D CUDA tensor (d, N)")
    if features.dtype not in (torch.float32, torch.float64):
        raise ValueError("features: expected float32 or float64")
    d, N = features.shape
    features = features.contiguous()
    y = _vec(target.reshape(-1), N, features.dtype, "target")
    if out is None:
        out = torch.empty(d, dtype=torch.float64, device=features.device)
    _vec(out, d, torch.float64, "out")          # validates the output vector
    prec = NLD_FP32 if features.dtype == torch.float32 else NLD_FP64
    fn = load().mis_scores_noalloc if noalloc else load().mis_scores
    _check(fn(ctypes.c_void_p(features.data_ptr()), N, d, y, prec, int(bins),
              ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def mis_scores_noalloc(features: torch.Tensor, target: torch.Tensor, bins: int = 0, stream=None,
                       out=None):
    """mis_scores_noalloc of nld.h: mis_scores on the library's static scratch."""
    return mis_scores(features, target, bins, stream, out=out, noalloc=True)


def mis_window_table(features: torch.Tensor, target: torch.Tensor, bins: int = 0, size: int = 3,
                     stream=None):
    """Windows from the mutual-information ranking (paper Sec. 5): features in decreasing score
    (ties by increasing index) cut into consecutive groups of `size`.  Returns (windows, scores)."""
    sc = mis_scores(features, target, bins, stream).cpu().tolist()
    order = sorted(range(len(sc)), key=lambda j: (-sc[j], j))
    return [order[k:k + size] for k in range(0, len(order), size)], sc


def pcg_solve_batched(plans, alphas, fs, us=None, tol: float = 1e-6, maxit: int = 500,
                      precond: bool = True, deflate: bool = True, use_u0: bool = False,
                      true_residual: bool = False, stream=None):
    """Solves (I + alpha_b L_b) u_b = f_b for every plan b together (see pcg_solve_batched in
    nld.h).  Returns (list of u_b, list of info dicts, status)."""
    n = len(plans)
    if not (len(alphas) == len(fs) == n) or n == 0:
        raise ValueError("plans, alphas and fs must have the same nonzero length")
    if us is None:
        us = [torch.empty_like(f) for f in fs]
    ph = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    al = (ctypes.c_double * n)(*[float(a) for a in alphas])
    fp = (ctypes.c_void_p * n)(*[_vec(f, p.N, p.dtype, "f").value for f, p in zip(fs, plans)])
    up = (ctypes.c_void_p * n)(*[_vec(u, p.N, p.dtype, "u").value for u, p in zip(us, plans)])
    opts = PcgOpts(float(tol), int(maxit), int(use_u0), _precond(precond), int(deflate),
                   int(true_residual), 0)
    infos = (PcgInfo * n)()
    st = load().pcg_solve_batched(ph, al, fp, up, n, ctypes.byref(opts), infos, _stream(stream))
    if st not in (NLD_OK, NLD_E_NOCONV, NLD_E_BREAKDOWN):
        _check(st)
    return us, [infos[b].as_dict() for b in range(n)], st


def adjoint_solve(plan: Plan, alpha, f, u, g, **kw):
    return plan.adjoint_solve(alpha, f, u, g, **kw)


class DenoiseSolve(torch.autograd.Function):
    """u = (I + alpha L(sigma, w))^-1 f with alpha = exp(log_alpha), sigma = exp(log_sigma).

    forward: nfft_plan + pcg_solve; backward: adjoint_solve (one adjoint solve with the same
    operator plus the sigma-derivative summation).  The features are data: no gradient flows
    into them; the gradient with respect to f is the adjoint state p.  log_alpha, log_sigma
    and weight are float64 CPU tensors; f is a GPU tensor of the plan's precision."""

    @staticmethod
    def forward(ctx, f, log_alpha, log_sigma, weight, features, windows, plan_kw, tol):
        L = len(windows)
        sig = torch.exp(log_sigma.detach()).tolist()
        wts = weight.detach().tolist()
        plan = Plan(features, windows, sig, wts, **plan_kw)
        alpha = float(torch.exp(log_alpha.detach()))
        u, info = plan.pcg_solve(alpha, f, tol=tol)
        if info["status"] != "OK":
            raise NldError(NLD_E_NOCONV, f"forward solve: {info}")
        ctx.plan, ctx.alpha, ctx.tol, ctx.L = plan, alpha, tol, L
        ctx.save_for_backward(f, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        f, u = ctx.saved_tensors
        p, grad, info = ctx.plan.adjoint_solve(ctx.alpha, f, u, grad_u.contiguous(), tol=ctx.tol)
        L = ctx.L
        g_la = torch.tensor(grad[0], dtype=torch.float64)
        g_ls = torch.tensor(grad[1:1 + L], dtype=torch.float64)
        g_w = torch.tensor(grad[1 + L:], dtype=torch.float64)
        ctx.plan.close()
        return p, g_la, g_ls, g_w, None, None, None, None
