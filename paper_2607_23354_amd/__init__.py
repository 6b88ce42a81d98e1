"""libmag: the weighting equation of metric magnitude on an MI355X (gfx950).

Python binding of the C ABI in ``include/mag.h``.  Tensors are PyTorch CUDA
(HIP) tensors; PyTorch supplies device memory and the stream, and every step
of the computation runs in the HIP library ``libmag.so``.

Problem (Section 2 of the paper): for points x_1..x_n in R^m and t > 0,
Z = exp[-t d] with d the Euclidean distance matrix; the weighting w solves
Z w = 1 and the magnitude is 1^T w.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import MagError, MagInfo, MagOpts, MagTplusInfo, MagTplusOpts  # noqa: F401

__all__ = ["Context", "weighting", "magnitude", "dmin", "zmatvec", "residual", "tile32",
           "factor32", "prec_apply", "factor64", "chol64_solve", "padded_size", "tplus", "dwdt", "dzmatvec",
           "MagnitudeFn", "weighting_and_magnitude", "weighting_batch", "tplus_batch",
           "eig_extremes", "weighting_zero", "MagError", "SOLVERS"]

SOLVERS = {"auto": _lib.MAG_AUTO, "fp64_dense": _lib.MAG_FP64_DENSE,
           "fp32_ir": _lib.MAG_FP32_IR, "hodlr": _lib.MAG_HODLR, "hss": _lib.MAG_HSS,
           "fp64_chol": _lib.MAG_FP64_CHOL}
SOLVER_NAMES = {v: k for k, v in SOLVERS.items()}
DIAG_BACKWARD = 1
DIAG_COND = 2


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _points(X: torch.Tensor) -> torch.Tensor:
    if X.dim() == 1:
        X = X[:, None]
    if X.dim() != 2 or X.dtype != torch.float64 or not X.is_cuda:
        raise ValueError("X must be a 2-D float64 CUDA tensor (n, m)")
    return X.contiguous()


class Context:
    """Owns a libmag context (device scratch memory) on one device."""

    def __init__(self, device: int | None = None):
        self.lib = _lib.load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        _lib.check(self.lib.mag_create(ctypes.byref(h), self.device), "mag_create")
        self.handle = h

    def set_workspace_limit(self, nbytes: int) -> None:
        """Cap the device memory this context may hold (0 = no cap); calls that
        would exceed it fail with MAG_ENOMEM."""
        _lib.check(self.lib.mag_set_workspace_limit(self.handle, int(nbytes)), "mag_set_workspace_limit")

    def set_spin_limit(self, polls: int) -> None:
        """Bound the sync-free triangular solves' waits (0 = the default); a
        call whose waits run out fails with MAG_EINTERNAL."""
        _lib.check(self.lib.mag_set_spin_limit(self.handle, int(polls)), "mag_set_spin_limit")

    def workspace_bytes(self) -> int:
        held = ctypes.c_uint64()
        _lib.check(self.lib.mag_workspace_bytes(self.handle, ctypes.byref(held)), "mag_workspace_bytes")
        return int(held.value)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.mag_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(self.lib.mag_set_stream(self.handle, ctypes.c_void_p(s)), "mag_set_stream")


_default: dict[int, Context] = {}


def _default_ctx(device: int) -> Context:
    c = _default.get(device)
    if c is None:
        c = _default[device] = Context(device)
    c._sync_stream()
    return c


def _ctx(ctx: Context | None, X: torch.Tensor) -> Context:
    if ctx is not None:
        ctx._sync_stream()
        return ctx
    dev = X.device.index if X.device.index is not None else torch.cuda.current_device()
    c = _default.get(dev)
    if c is None:
        c = _default[dev] = Context(dev)
    c._sync_stream()
    return c


def make_opts(solver: str = "auto", tol: float = 1e-12, max_outer: int | None = None,
              gmres_restart: int | None = None, max_gmres: int | None = None,
              inner_tol: float | None = None, profile: bool = False, leaf: int | None = None,
              max_rank: int | None = None, oversample: int | None = None,
              seed: int | None = None, inner_prec: str = "fp64", diag: int = 0,
              power_iters: int | None = None) -> MagOpts:
    o = MagOpts()
    _lib.load().mag_opts_default(ctypes.byref(o))
    o.solver = SOLVERS[solver]
    o.tol = tol
    if max_outer is not None:
        o.max_outer = max_outer
    if gmres_restart is not None:
        o.gmres_restart = gmres_restart
    if max_gmres is not None:
        o.max_gmres = max_gmres
    if inner_tol is not None:
        o.inner_tol = inner_tol
    if leaf is not None:
        o.leaf = leaf
    if max_rank is not None:
        o.max_rank = max_rank
    if oversample is not None:
        o.oversample = oversample
    if seed is not None:
        o.seed = seed
    o.profile = 1 if profile else 0
    if inner_prec not in ("fp64", "fp32"):
        raise ValueError(f"inner_prec must be 'fp64' or 'fp32', not {inner_prec!r}")
    o.inner_prec = 0 if inner_prec == "fp64" else 1
    o.diag = int(diag)
    if power_iters is not None:
        o.power_iters = power_iters
    return o


@dataclass
class Result:
    w: torch.Tensor
    info: dict


def weighting(X: torch.Tensor, t: float, *, ctx: Context | None = None, out: torch.Tensor | None = None,
              raise_on_noconv: bool = True, **opts) -> Result:
    """Solve Z w = 1 (eq. weighting) on the device; returns w and the info
    record (iterations, residual, magnitude, min w, phase times)."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    w = out if out is not None else torch.empty(n, dtype=torch.float64, device=X.device)
    o = make_opts(**opts)
    info = MagInfo()
    rc = c.lib.mag_weighting(c.handle, _ptr(X), n, m, float(t), _ptr(w), ctypes.byref(o), ctypes.byref(info))
    if rc != _lib.MAG_OK and not (rc == _lib.MAG_ENOCONV and not raise_on_noconv):
        raise MagError(rc, "mag_weighting")
    return Result(w, info.as_dict())


def weighting_zero(X: torch.Tensor, *, ctx: Context | None = None, out: torch.Tensor | None = None,
                   raise_on_noconv: bool = True, **opts) -> Result:
    """Weighting at scale zero (eq. scaleZero): w0 = d^{-1} 1 / (1^T d^{-1} 1),
    the limit of w as t -> 0, from the positive definite c 1 1^T - d.  info also
    holds sum_dinv = 1^T d^{-1} 1 and c."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    w = out if out is not None else torch.empty(n, dtype=torch.float64, device=X.device)
    o = make_opts(**opts)
    info = MagInfo()
    sd, cu = ctypes.c_double(), ctypes.c_double()
    rc = c.lib.mag_weighting_zero(c.handle, _ptr(X), n, m, _ptr(w), ctypes.byref(o), ctypes.byref(info),
                                  ctypes.byref(sd), ctypes.byref(cu))
    if rc != _lib.MAG_OK and not (rc == _lib.MAG_ENOCONV and not raise_on_noconv):
        raise MagError(rc, "mag_weighting_zero")
    d = info.as_dict()
    d["sum_dinv"], d["c"], d["status"] = sd.value, cu.value, rc
    return Result(w, d)


def magnitude(X: torch.Tensor, t: float, *, ctx: Context | None = None, **opts) -> float:
    """Mag = 1^T w (Section 2)."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    o = make_opts(**opts)
    M = ctypes.c_double()
    _lib.check(c.lib.mag_magnitude(c.handle, _ptr(X), n, m, float(t), ctypes.byref(M), None,
                                   ctypes.byref(o), None), "mag_magnitude")
    return M.value


def dmin(X: torch.Tensor, *, ctx: Context | None = None) -> float:
    """min_{j != k} ||x_j - x_k||, brute force on the device."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    d = ctypes.c_double()
    _lib.check(c.lib.mag_dmin(c.handle, _ptr(X), n, m, ctypes.byref(d)), "mag_dmin")
    return d.value


def padded_size(n: int) -> int:
    return int(_lib.load().mag_padded_size(n))


def zmatvec(X: torch.Tensor, t: float, v: torch.Tensor, *, ctx: Context | None = None) -> torch.Tensor:
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    v = v.contiguous()
    y = torch.empty(n, dtype=torch.float64, device=X.device)
    _lib.check(c.lib.mag_zmatvec(c.handle, _ptr(X), n, m, float(t), _ptr(v), _ptr(y)), "mag_zmatvec")
    return y


def residual(X: torch.Tensor, t: float, w: torch.Tensor, *, ctx: Context | None = None):
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    w = w.contiguous()
    r = torch.empty(n, dtype=torch.float64, device=X.device)
    rinf = ctypes.c_double()
    _lib.check(c.lib.mag_residual(c.handle, _ptr(X), n, m, float(t), _ptr(w), _ptr(r), ctypes.byref(rinf)),
               "mag_residual")
    return r, rinf.value


def tile32(X: torch.Tensor, t: float, *, ctx: Context | None = None) -> torch.Tensor:
    """FP32 Z as the tile generator writes it (npad x npad, column-major:
    the returned tensor A satisfies A[j, i] = Z_ij)."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    npad = padded_size(n)
    A = torch.zeros((npad, npad), dtype=torch.float32, device=X.device)
    _lib.check(c.lib.mag_tile32(c.handle, _ptr(X), n, m, float(t), _ptr(A)), "mag_tile32")
    return A


def factor32(X: torch.Tensor, t: float, shift: float = 0.0, *, ctx: Context | None = None):
    """FP32 Cholesky factor (column-major npad x npad buffer, lower triangle
    valid) and the inverses of its 128-diagonal blocks."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    npad = padded_size(n)
    L = torch.zeros((npad, npad), dtype=torch.float32, device=X.device)
    dinv = torch.zeros((npad // 128, 128, 128), dtype=torch.float32, device=X.device)
    bd = ctypes.c_int32()
    _lib.check(c.lib.mag_factor32(c.handle, _ptr(X), n, m, float(t), float(shift), _ptr(L), _ptr(dinv),
                                  ctypes.byref(bd)), "mag_factor32")
    return L, dinv, int(bd.value)


def prec_apply(L: torch.Tensor, dinv: torch.Tensor, n: int, r: torch.Tensor, *,
               ctx: Context | None = None) -> torch.Tensor:
    c = _ctx(ctx, r)
    r = r.contiguous()
    z = torch.empty(n, dtype=torch.float64, device=r.device)
    _lib.check(c.lib.mag_prec_apply(c.handle, _ptr(L), _ptr(dinv), n, _ptr(r), _ptr(z)), "mag_prec_apply")
    return z


def factor64(X: torch.Tensor, t: float, *, ctx: Context | None = None):
    """FP64 Cholesky factor of the fp64_chol solver (column-major npad x npad
    buffer: L in the lower triangle, L^T in the upper one) and the inverses of
    its 64-diagonal blocks."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    npad = padded_size(n)
    L = torch.zeros((npad, npad), dtype=torch.float64, device=X.device)
    dinv = torch.zeros((npad // 64, 64, 64), dtype=torch.float64, device=X.device)
    bd = ctypes.c_int32()
    _lib.check(c.lib.mag_factor64(c.handle, _ptr(X), n, m, float(t), _ptr(L), _ptr(dinv), ctypes.byref(bd)),
               "mag_factor64")
    return L, dinv, int(bd.value)


def chol64_solve(L: torch.Tensor, dinv: torch.Tensor, n: int, r: torch.Tensor, *,
                 ctx: Context | None = None) -> torch.Tensor:
    """z = (L L^T)^{-1} r with the factor of factor64."""
    c = _ctx(ctx, r)
    r = r.contiguous()
    z = torch.empty(n, dtype=torch.float64, device=r.device)
    _lib.check(c.lib.mag_chol64_solve(c.handle, _ptr(L), _ptr(dinv), n, _ptr(r), _ptr(z)), "mag_chol64_solve")
    return z


def dzmatvec(X: torch.Tensor, t: float, v: torch.Tensor, *, ctx: Context | None = None) -> torch.Tensor:
    """(D o Z) v with (D o Z)_jk = d_jk exp(-t d_jk), matrix-free FP64."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    v = v.contiguous()
    y = torch.empty(n, dtype=torch.float64, device=X.device)
    _lib.check(c.lib.mag_dzmatvec(c.handle, _ptr(X), n, m, float(t), _ptr(v), _ptr(y)), "mag_dzmatvec")
    return y


def dwdt(X: torch.Tensor, t: float, *, ctx: Context | None = None, **opts):
    """(w, dw/dt) at scale t, dw/dt = Z^{-1} (D o Z) w."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    o = make_opts(**opts)
    w = torch.empty(n, dtype=torch.float64, device=X.device)
    d = torch.empty(n, dtype=torch.float64, device=X.device)
    _lib.check(c.lib.mag_dwdt(c.handle, _ptr(X), n, m, float(t), _ptr(w), _ptr(d), ctypes.byref(o)), "mag_dwdt")
    return w, d


def eig_extremes(X: torch.Tensor, t: float, *, v0: torch.Tensor | None = None, max_iter: int = 80,
                 rtol: float = 1e-8, ctx: Context | None = None, **opts) -> dict:
    """Extreme eigenvalues of Z(t) by symmetric Lanczos (Section 4.2's
    positive-definiteness check): lambda_max from Z's matrix-free products,
    lambda_min from Z^{-1} through the FP32 factor + refinement.  Returns the
    info fields as a dict (status: MAG_OK, or MAG_ENOCONV when an inner solve
    missed its tolerance)."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    o = make_opts(**opts)
    eo = _lib.MagEigOpts()
    c.lib.mag_eig_opts_default(ctypes.byref(eo))
    eo.max_iter, eo.rtol = int(max_iter), float(rtol)
    if v0 is not None:
        if v0.device != X.device or v0.dtype != torch.float64 or v0.numel() != n:
            raise ValueError("v0: float64 vector of n entries on the device of X")
        v0 = v0.contiguous()
    info = _lib.MagEigInfo()
    rc = c.lib.mag_eig_extremes(c.handle, _ptr(X), n, m, float(t), _ptr(v0), ctypes.byref(eo), ctypes.byref(o),
                                ctypes.byref(info))
    if rc not in (_lib.MAG_OK, _lib.MAG_ENOCONV):
        _lib.check(rc, "mag_eig_extremes")
    d = info.as_dict()
    d["status"] = rc
    return d


@dataclass
class TplusResult:
    t_plus: float
    w: torch.Tensor | None
    info: dict


TPLUS_METHODS = {"bisection": 0, "ridders": 1}


def _tplus_method(method: str) -> int:
    if method not in TPLUS_METHODS:
        raise ValueError(f"method must be one of {sorted(TPLUS_METHODS)}")
    return TPLUS_METHODS[method]


def tplus(X: torch.Tensor, *, ctx: Context | None = None, grid: int = 32, lo_factor: float = 1e-3,
          rtol: float = 1e-6, newton: bool = True, max_extend: int = 2, eps: float = 0.0,
          t_lo: float = 0.0, t_hi: float = 0.0, want_w: bool = True, method: str = "bisection",
          **opts) -> TplusResult:
    """Cutoff t_+ (least t from which w >= 0) by a downward log-grid scan from
    log(n-1)/d_min, then the bracket refined in log t by safeguarded
    Newton/bisection (method "bisection") or Ridders' method ("ridders")."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    to = MagTplusOpts()
    c.lib.mag_tplus_opts_default(ctypes.byref(to))
    to.grid, to.lo_factor, to.rtol, to.newton = grid, lo_factor, rtol, 1 if newton else 0
    to.max_extend, to.eps, to.t_lo, to.t_hi = max_extend, eps, t_lo, t_hi
    to.method = _tplus_method(method)
    o = make_opts(**opts)
    w = torch.empty(n, dtype=torch.float64, device=X.device) if want_w else None
    tp = ctypes.c_double()
    info = MagTplusInfo()
    _lib.check(c.lib.mag_tplus(c.handle, _ptr(X), n, m, ctypes.byref(to), ctypes.byref(o), ctypes.byref(tp),
                               _ptr(w), ctypes.byref(info)), "mag_tplus")
    return TplusResult(tp.value, w if (want_w and not info.no_sign_change) else None, info.as_dict())


class _FactorHandle:
    """Owns a mag_factor (the FP32 factor kept by the forward pass)."""

    def __init__(self, lib, handle):
        self.lib, self.handle = lib, handle

    def __del__(self):
        if self.handle:
            self.lib.mag_factor_free(self.handle)
            self.handle = None


class MagnitudeFn(torch.autograd.Function):
    """(w, Mag) = MagnitudeFn.apply(X, t) with a hand-written adjoint.

    Forward: mag_weighting_fwd (FP32 MFMA factor + FP64 refinement), keeping
    the factor.  Backward: mag_weighting_vjp, which reuses the factor for
    lambda = Z^{-1}(gM 1 + gw) and makes one matrix-free FP64 pass for
    dL/dt = lambda^T (D o Z) w and dL/dX."""

    @staticmethod
    def forward(fctx, X, t):
        X = _points(X)
        n, m = X.shape
        c = _ctx(None, X)
        tval = float(t)
        o = make_opts()
        info = MagInfo()
        w = torch.empty(n, dtype=torch.float64, device=X.device)
        h = ctypes.c_void_p()
        _lib.check(c.lib.mag_weighting_fwd(c.handle, _ptr(X), n, m, tval, _ptr(w), ctypes.byref(h),
                                           ctypes.byref(o), ctypes.byref(info)), "mag_weighting_fwd")
        fctx.factor = _FactorHandle(c.lib, h)
        fctx.tval = tval
        fctx.t_is_tensor = isinstance(t, torch.Tensor)
        fctx.set_materialize_grads(False)
        fctx.save_for_backward(X, w)
        M = torch.tensor(info.magnitude, dtype=torch.float64, device=X.device)
        return w, M

    @staticmethod
    def backward(fctx, gw, gM):
        X, w = fctx.saved_tensors
        n, m = X.shape
        c = _ctx(None, X)
        gMv = float(gM) if gM is not None else 0.0
        gwp = None
        if gw is not None:
            gw = gw.contiguous().to(torch.float64)
            gwp = _ptr(gw)
        need_x = fctx.needs_input_grad[0]
        need_t = fctx.needs_input_grad[1]
        dX = torch.empty((n, m), dtype=torch.float64, device=X.device) if need_x else None
        dt = ctypes.c_double()
        o = make_opts()
        _lib.check(c.lib.mag_weighting_vjp(c.handle, fctx.factor.handle, _ptr(X), n, m, fctx.tval, _ptr(w),
                                           gMv, gwp, _ptr(dX), ctypes.byref(dt) if need_t else None,
                                           ctypes.byref(o)), "mag_weighting_vjp")
        gt = None
        if need_t and fctx.t_is_tensor:
            gt = torch.tensor(dt.value, dtype=torch.float64, device=X.device)
        return dX, gt


def weighting_and_magnitude(X: torch.Tensor, t):
    """Differentiable (w, Mag) of eq. weighting (see MagnitudeFn)."""
    return MagnitudeFn.apply(X, t)


def _pack(X: torch.Tensor, offs):
    X = _points(X)
    offs = [int(o) for o in offs]
    arr = (ctypes.c_int64 * len(offs))(*offs)
    return X, offs, arr


def weighting_batch(X: torch.Tensor, offs, t, *, ctx: Context | None = None, raise_on_noconv: bool = True,
                    **opts):
    """Batched weightings: cloud b is rows [offs[b], offs[b+1]) of X, solved at
    scale t[b].  Returns (w packed like X, magnitudes list, info list)."""
    X, offs, arr = _pack(X, offs)
    B = len(offs) - 1
    n, m = X.shape
    c = _ctx(ctx, X)
    tt = (ctypes.c_double * B)(*[float(v) for v in t])
    Ms = (ctypes.c_double * B)()
    infos = (MagInfo * B)()
    w = torch.empty(offs[-1] - offs[0], dtype=torch.float64, device=X.device)
    o = make_opts(**opts)
    rc = c.lib.mag_weighting_batch(c.handle, B, _ptr(X), arr, m, tt, _ptr(w), Ms, ctypes.byref(o), infos)
    if rc != _lib.MAG_OK and not (rc == _lib.MAG_ENOCONV and not raise_on_noconv):
        raise MagError(rc, "mag_weighting_batch")
    return w, list(Ms), [i.as_dict() for i in infos]


def tplus_batch(X: torch.Tensor, offs, *, ctx: Context | None = None, grid: int = 32, lo_factor: float = 1e-3,
                rtol: float = 1e-6, newton: bool = True, max_extend: int = 2, eps: float = 0.0,
                want_w: bool = False, method: str = "bisection", **opts):
    """Batched cutoff search over the clouds rows [offs[b], offs[b+1]) of X.
    Returns (t_plus list, w packed or None, info list)."""
    X, offs, arr = _pack(X, offs)
    B = len(offs) - 1
    n, m = X.shape
    c = _ctx(ctx, X)
    to = MagTplusOpts()
    c.lib.mag_tplus_opts_default(ctypes.byref(to))
    to.grid, to.lo_factor, to.rtol, to.newton = grid, lo_factor, rtol, 1 if newton else 0
    to.max_extend, to.eps = max_extend, eps
    to.method = _tplus_method(method)
    o = make_opts(**opts)
    tp = (ctypes.c_double * B)()
    infos = (MagTplusInfo * B)()
    w = torch.zeros(offs[-1] - offs[0], dtype=torch.float64, device=X.device) if want_w else None
    _lib.check(c.lib.mag_tplus_batch(c.handle, B, _ptr(X), arr, m, ctypes.byref(to), ctypes.byref(o), tp,
                                     _ptr(w), infos), "mag_tplus_batch")
    return list(tp), w, [i.as_dict() for i in infos]


def tune_panel(n: int, nb: int, *, ctx: Context | None = None, device: int = 0) -> None:
    """Panel width (256 or 512; 0 = built-in) of the FP32 factor for n's size bucket."""
    c = ctx if ctx is not None else _default_ctx(device)
    _lib.check(c.lib.mag_tune_panel(c.handle, int(n), int(nb)), "mag_tune_panel")


def autotune(X: torch.Tensor, t: float, *, reps: int = 2, ctx: Context | None = None):
    """Time the FP32 factor of this problem with panel widths 256 and 512 and
    keep the faster for its size bucket; returns (width, (ms_256, ms_512))."""
    X = _points(X)
    n, m = X.shape
    c = _ctx(ctx, X)
    nb = ctypes.c_int32(0)
    ms = (ctypes.c_double * 2)()
    _lib.check(c.lib.mag_autotune(c.handle, _ptr(X), n, m, float(t), int(reps), ctypes.byref(nb), ms), "mag_autotune")
    return nb.value, (ms[0], ms[1])


def tune_batch_group(max_n: int, group: int, *, ctx: Context | None = None, device: int = 0) -> None:
    """Panel grouping of the batched factorisation for max_n's size bucket:
    1 single 256-column panels, 2 pairs, 0 the built-in choice (pairs)."""
    c = ctx if ctx is not None else _default_ctx(device)
    _lib.check(c.lib.mag_tune_batch_group(c.handle, int(max_n), int(group)), "mag_tune_batch_group")


def autotune_batch(X: torch.Tensor, offs, t, *, reps: int = 2, ctx: Context | None = None):
    """Time the batched factorisation of these clouds with single panels and
    with pairs and keep the faster for the bucket of the largest cloud;
    returns (group, (ms_single, ms_pairs))."""
    X, offs, arr = _pack(X, offs)
    B = len(offs) - 1
    n, m = X.shape
    c = _ctx(ctx, X)
    tt = (ctypes.c_double * B)(*[float(v) for v in t])
    g = ctypes.c_int32(0)
    ms = (ctypes.c_double * 2)()
    _lib.check(c.lib.mag_autotune_batch(c.handle, B, _ptr(X), arr, m, tt, int(reps), ctypes.byref(g), ms),
               "mag_autotune_batch")
    return g.value, (ms[0], ms[1])


def tune_save(path: str, *, ctx: Context | None = None, device: int = 0) -> None:
    c = ctx if ctx is not None else _default_ctx(device)
    _lib.check(c.lib.mag_tune_save(c.handle, os.fsencode(path)), "mag_tune_save")


def tune_load(path: str, *, ctx: Context | None = None, device: int = 0) -> None:
    c = ctx if ctx is not None else _default_ctx(device)
    _lib.check(c.lib.mag_tune_load(c.handle, os.fsencode(path)), "mag_tune_load")
