"""CPU oracle for the weighting equation Z w = 1 of metric magnitude.

TEST INFRASTRUCTURE ONLY.  Plain FP64 reference used by the test-suite, the
smoke check and the benchmark's CPU-baseline leg; never by the library.  It
shares no code with the HIP path and does not import it.

The arithmetic lives in ``mag_oracle.c`` (plain C, every operation rounded as
written); this module wraps it with ctypes and adds the steps that are plain
Python on top of it: the t_+ search by bisection, the condition estimate and
the gradient assembly.

Paper passages followed (Huntsman et al., "Scalably computing metric
magnitude"):
  * Section 2: Z = exp[-t d] with Euclidean d; weighting Z w = 1
    (eq. weighting); magnitude Mag = 1^T w; w unique as Z is positive
    definite.
  * Section 2, cutoff paragraph and its footnote: t_+ is the least t with
    w >= 0, found by root-finding on min_j w_j, bracketed by
    t_+ <= log(n-1)/min d; halt early when min w lies in (0, eps).
  * Appendix A: the cutoff computed by binary search.
  * Section 4.2: positive definiteness checked by a Cholesky attempt and an
    extreme-eigenvalue estimate.
  * Appendix C.1, eq. scaleZero: the weighting at scale zero,
    lim_{t -> 0} Z(t)^{-1} 1 = d^{-1} 1 / (1^T d^{-1} 1); d is indefinite, so
    d u = 1 is solved by Gaussian elimination with partial pivoting.

Readings where the paper is silent (each listed in the design notes):
  * t_+ := inf{t > 0 : w(s) >= 0 for all s >= t}; located as the largest
    sign change on a log grid scanned downward from the bound.
  * grid: ``grid`` points log-spaced on [t_b * lo_factor, t_b]; extended
    downward by lo_factor up to ``max_extend`` times when w >= 0 on it.
  * bisection at the geometric midpoint until (t_hi - t_lo)/t_hi <= rtol;
    the returned t_+ is t_hi, where min w >= 0.
  * eps of the early halt = n * 2^-53.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mag_oracle.c")
_SO = os.path.join(_HERE, "libmag_oracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile mag_oracle.c into libmag_oracle.so with gcc (OpenMP, no
    contraction, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_SO)
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_dist.restype = ctypes.c_double
        L.orc_dist.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_int64, ctypes.c_int64]
        L.orc_distance_matrix.argtypes = [_D, ctypes.c_int64, ctypes.c_int, _D]
        L.orc_zmatrix.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_double, _D]
        L.orc_dmin.restype = ctypes.c_double
        L.orc_dmin.argtypes = [_D, ctypes.c_int64, ctypes.c_int]
        L.orc_cholesky.restype = ctypes.c_int
        L.orc_cholesky.argtypes = [_D, ctypes.c_int64]
        L.orc_chol_solve.argtypes = [_D, ctypes.c_int64, _D, _D]
        L.orc_residual.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_double, _D,
                                   _I64, ctypes.c_int64, _D]
        L.orc_residual_rhs.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_double, _D, _D,
                                       _I64, ctypes.c_int64, _D]
        L.orc_solve_refine.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_double, _D, _D,
                                       ctypes.c_int, _D, _D]
        L.orc_zmatvec.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_double, _D, _D]
        L.orc_dzmatvec.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_double, _D, _D]
        L.orc_grad_x.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_double, _D, _D, _D]
        L.orc_grad_x_rows.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_double, _D, _D, _I64,
                                      ctypes.c_int64, _D]
        L.orc_sum.restype = ctypes.c_double
        L.orc_sum.argtypes = [_D, ctypes.c_int64]
        L.orc_dist_residual.argtypes = [_D, ctypes.c_int64, ctypes.c_int, _D, _I64, ctypes.c_int64, _D]
        L.orc_dist_solve_ones.restype = ctypes.c_int
        L.orc_dist_solve_ones.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _D, _D]
        L.orc_weighting.restype = ctypes.c_int
        L.orc_weighting.argtypes = [_D, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                    _D, _D, _D]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _pts(X) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    return X


def num_threads() -> int:
    return int(lib().orc_num_threads())


class NotPositiveDefinite(RuntimeError):
    pass


# --------------------------------------------------------------------------
# Elementwise pieces
# --------------------------------------------------------------------------

def distance_matrix(X) -> np.ndarray:
    """d_jk = ||x_j - x_k|| (Section 2), exact differences."""
    X = _pts(X)
    n, m = X.shape
    D = np.empty((n, n))
    lib().orc_distance_matrix(_p(X), n, m, _p(D))
    return D


def zmatrix(X, t: float) -> np.ndarray:
    """Z = exp[-t d] (Section 2)."""
    X = _pts(X)
    n, m = X.shape
    Z = np.empty((n, n))
    lib().orc_zmatrix(_p(X), n, m, float(t), _p(Z))
    return Z


def dmin(X) -> float:
    """min over j != k of d_jk, brute force (the bound's denominator)."""
    X = _pts(X)
    n, m = X.shape
    return float(lib().orc_dmin(_p(X), n, m))


def t_bound(X) -> float:
    """t_b = log(n-1)/min d, the upper bound on t_+ (Sections 1 and 2)."""
    X = _pts(X)
    return float(np.log(X.shape[0] - 1) / dmin(X))


def cholesky(A) -> np.ndarray:
    """Lower Cholesky factor (plain column-by-column form); raises
    NotPositiveDefinite on a non-positive pivot."""
    L = np.array(A, dtype=np.float64, order="C", copy=True)
    n = L.shape[0]
    st = lib().orc_cholesky(_p(L), n)
    if st != 0:
        raise NotPositiveDefinite(f"pivot {st - 1} not positive")
    return np.tril(L)


def chol_solve(L, b) -> np.ndarray:
    L = np.ascontiguousarray(L, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty_like(b)
    lib().orc_chol_solve(_p(L), L.shape[0], _p(b), _p(x))
    return x


def residual(X, t: float, w, rows=None, b=None) -> np.ndarray:
    """r = 1 - Z w (or b - Z w for a given right-hand side b) with Z
    regenerated from X, accumulated with Dot2 (compensated: as if computed in
    doubled precision).  ``rows`` selects a subset of rows."""
    X = _pts(X)
    n, m = X.shape
    w = np.ascontiguousarray(w, dtype=np.float64)
    if b is not None:
        b = np.ascontiguousarray(b, dtype=np.float64)
        if b.shape != (n,):
            raise ValueError("b must have one entry per point")
        if rows is None:
            r = np.empty(n)
            lib().orc_residual_rhs(_p(X), n, m, float(t), _p(b), _p(w), None, 0, _p(r))
        else:
            rows = np.ascontiguousarray(rows, dtype=np.int64)
            r = np.empty(len(rows))
            lib().orc_residual_rhs(_p(X), n, m, float(t), _p(b), _p(w), rows.ctypes.data_as(_I64),
                                   len(rows), _p(r))
        return r
    if rows is None:
        r = np.empty(n)
        lib().orc_residual(_p(X), n, m, float(t), _p(w), None, 0, _p(r))
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        r = np.empty(len(rows))
        lib().orc_residual(_p(X), n, m, float(t), _p(w), rows.ctypes.data_as(_I64), len(rows), _p(r))
    return r


def zmatvec(X, t: float, v) -> np.ndarray:
    X = _pts(X)
    n, m = X.shape
    v = np.ascontiguousarray(v, dtype=np.float64)
    y = np.empty(n)
    lib().orc_zmatvec(_p(X), n, m, float(t), _p(v), _p(y))
    return y


def dzmatvec(X, t: float, v) -> np.ndarray:
    """(D o Z) v, i.e. -(dZ/dt) v."""
    X = _pts(X)
    n, m = X.shape
    v = np.ascontiguousarray(v, dtype=np.float64)
    y = np.empty(n)
    lib().orc_dzmatvec(_p(X), n, m, float(t), _p(v), _p(y))
    return y


def msum(v) -> float:
    """Compensated (Neumaier) sum."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    return float(lib().orc_sum(_p(v), len(v)))


# --------------------------------------------------------------------------
# Weighting and magnitude (eq. weighting)
# --------------------------------------------------------------------------

class Weighting:
    """Result of the oracle solve: w (refined), w_plain (no refinement), the
    factor L (lower, row-major), M = 1^T w and min/argmin of w."""

    def __init__(self, X, t, w, w_plain, L):
        self.X, self.t, self.w, self.w_plain, self.L = X, t, w, w_plain, L
        self.M = msum(w)
        self.argmin = int(np.argmin(w))
        self.min_w = float(w[self.argmin])

    def solve(self, b, refine: int = 2):
        """Z^{-1} b with the stored factor plus refinement steps whose
        residuals b - Z x are Dot2 sums started from b (never through 1 - Z x,
        which would round away the compensated part when b != 1)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        n, m = self.X.shape
        x = np.empty(n)
        lib().orc_solve_refine(_p(self.X), n, m, float(self.t), _p(self.L), _p(b), int(refine), None, _p(x))
        return x


def weighting(X, t: float, refine: int = 3) -> Weighting:
    """Solve Z w = 1 in FP64: Z from X, plain Cholesky, forward/back solve,
    then ``refine`` steps of refinement with Dot2 residuals."""
    X = _pts(X)
    n, m = X.shape
    if not (t > 0 and np.isfinite(t)):
        raise ValueError("t must be positive and finite")
    work = np.empty((n, n))
    w = np.empty(n)
    wp = np.empty(n)
    st = lib().orc_weighting(_p(X), n, m, float(t), int(refine), _p(wp), _p(w), _p(work))
    if st != 0:
        raise NotPositiveDefinite(f"Z not numerically positive definite (pivot {st - 1})")
    return Weighting(X, float(t), w, wp, work)


def magnitude(X, t: float) -> float:
    """Mag = 1^T w (Section 2)."""
    return weighting(X, t).M


# --------------------------------------------------------------------------
# Weighting at scale zero (Appendix C.1, eq. scaleZero)
# --------------------------------------------------------------------------

def weighting_zero(X, refine: int = 2):
    """(w0, sum_dinv): w0 = d^{-1} 1 / (1^T d^{-1} 1), the limit of the
    weighting as t -> 0, and 1^T d^{-1} 1.  d u = 1 by LU with partial
    pivoting and ``refine`` Dot2-residual refinement steps; the sum is
    compensated.  One point: w0 = 1 (the limit of Z(t)^{-1} 1 = 1) and
    sum_dinv = inf (d = 0)."""
    X = _pts(X)
    n, m = X.shape
    if n == 1:
        return np.ones(1), float("inf")
    u = np.empty(n)
    work = np.empty((n, n))
    st = lib().orc_dist_solve_ones(_p(X), n, m, int(refine), _p(u), _p(work))
    if st != 0:
        raise NotPositiveDefinite(f"d singular (column {st - 1}): coincident points")
    s = msum(u)
    return u / s, s


def dist_residual(X, u, rows=None) -> np.ndarray:
    """r = 1 - d u (Dot2), on all rows or the given ones."""
    X = _pts(X)
    n, m = X.shape
    u = np.ascontiguousarray(u, dtype=np.float64)
    if rows is None:
        r = np.empty(n)
        lib().orc_dist_residual(_p(X), n, m, _p(u), None, 0, _p(r))
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        r = np.empty(len(rows))
        lib().orc_dist_residual(_p(X), n, m, _p(u), rows.ctypes.data_as(_I64), len(rows), _p(r))
    return r


# --------------------------------------------------------------------------
# Conditioning (Section 4.2 sanity check; acceptance domain of the tests)
# --------------------------------------------------------------------------

def cond_estimate(sol: Weighting, iters: int = 200, seed: int = 12345, rtol: float = 1e-10):
    """(lambda_max, lambda_min, cond) of Z: power iteration with Z for
    lambda_max, inverse iteration through the factor for lambda_min
    (Rayleigh quotients; each side stops when its estimate changes by at most
    rtol relative, or after ``iters`` steps)."""
    X, t = sol.X, sol.t
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    lmax = 0.0
    for _ in range(iters):
        y = zmatvec(X, t, v)
        lmax_new = float(v @ y)
        v = y / np.linalg.norm(y)
        if abs(lmax_new - lmax) <= rtol * abs(lmax_new):
            lmax = lmax_new
            break
        lmax = lmax_new
    u = rng.standard_normal(n)
    u /= np.linalg.norm(u)
    mu = np.inf
    for _ in range(iters):
        y = chol_solve(sol.L, u)
        mu_new = float(u @ y)  # approx 1/lambda_min
        u = y / np.linalg.norm(y)
        if abs(mu_new - mu) <= rtol * abs(mu_new):
            mu = mu_new
            break
        mu = mu_new
    lmin = 1.0 / mu
    return lmax, lmin, lmax / lmin


def kappa_M(sol: Weighting) -> float:
    """|w|^T Z |w| / |M|: first-order sensitivity of M to componentwise
    relative perturbations of Z."""
    aw = np.abs(sol.w)
    return float(aw @ zmatvec(sol.X, sol.t, aw) / abs(sol.M))


# --------------------------------------------------------------------------
# Gradients (differentiating eq. weighting)
# --------------------------------------------------------------------------

def grad(X, t: float, gM: float = 1.0, gw=None, sol: Weighting | None = None):
    """Vector-Jacobian product of (w, M) = (Z^{-1} 1, 1^T w) at (X, t).

    With lambda = Z^{-1}(gM 1 + gw):
        dL/dt   = lambda^T (D o Z) w
        dL/dx_j = t sum_{k != j} (lambda_j w_k + lambda_k w_j) Z_jk (x_j - x_k)/d_jk
    Returns (dL/dt, dL/dX (n x m), sol)."""
    X = _pts(X)
    n, m = X.shape
    if sol is None:
        sol = weighting(X, t)
    g = np.full(n, float(gM))
    if gw is not None:
        g = g + np.asarray(gw, dtype=np.float64)
        lam = sol.solve(g)
    else:
        lam = float(gM) * sol.w
    dt = float(lam @ dzmatvec(X, t, sol.w))
    dX = np.empty((n, m))
    lib().orc_grad_x(_p(X), n, m, float(t), _p(np.ascontiguousarray(lam)), _p(sol.w), _p(dX))
    return dt, dX, sol


def grad_x_rows(X, t: float, lam, w, rows) -> np.ndarray:
    """Rows of dL/dX = t sum_{k != j} (lambda_j w_k + lambda_k w_j) Z_jk (x_j - x_k)/d_jk
    for given lambda and w (one output row at a time)."""
    X = _pts(X)
    n, m = X.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((len(rows), m))
    lib().orc_grad_x_rows(_p(X), n, m, float(t), _p(np.ascontiguousarray(lam, dtype=np.float64)),
                          _p(np.ascontiguousarray(w, dtype=np.float64)), rows.ctypes.data_as(_I64),
                          len(rows), _p(out))
    return out


def dw_dt(sol: Weighting) -> np.ndarray:
    """dw/dt = Z^{-1} (D o Z) w."""
    return sol.solve(dzmatvec(sol.X, sol.t, sol.w))


# --------------------------------------------------------------------------
# Cutoff t_+ (Section 2 cutoff paragraph; Appendix A binary search)
# --------------------------------------------------------------------------

class TPlus:
    def __init__(self, t_plus, t_bound, d_min, min_w, solves, no_sign_change, bracket):
        self.t_plus = t_plus
        self.t_bound = t_bound
        self.d_min = d_min
        self.min_w = min_w
        self.solves = solves
        self.no_sign_change = no_sign_change
        self.bracket = bracket


def min_w(X, t: float) -> float:
    return weighting(X, t).min_w


def tplus(X, grid: int = 32, lo_factor: float = 1e-3, rtol: float = 1e-6,
          max_extend: int = 2, eps: float | None = None) -> TPlus:
    """Cutoff t_+ by a downward scan of a log grid from the bound, then
    bisection (geometric midpoint) on the bracketing cell."""
    X = _pts(X)
    n = X.shape[0]
    dm = dmin(X)
    if n <= 2:
        return TPlus(0.0, np.inf if n < 2 else float(np.log(max(n - 1, 1)) / dm), dm, 1.0, 0, True, None)
    tb = float(np.log(n - 1) / dm)
    if eps is None:
        eps = n * 2.0 ** -53
    solves = 0
    hi_t, hi_min = None, None
    lo_t = None
    top = tb
    for ext in range(max_extend + 1):
        ts = np.geomspace(top * lo_factor, top, grid)
        for t in ts[::-1]:
            if hi_t is not None and t >= hi_t:
                continue
            mw = min_w(X, t)
            solves += 1
            if mw < 0.0:
                lo_t = float(t)
                break
            hi_t, hi_min = float(t), mw
        if lo_t is not None:
            break
        top = top * lo_factor
    if lo_t is None:
        return TPlus(0.0, tb, dm, hi_min, solves, True, None)
    lo, hi = lo_t, hi_t
    while (hi - lo) / hi > rtol:
        mid = float(np.sqrt(lo * hi))
        mw = min_w(X, mid)
        solves += 1
        if mw < 0.0:
            lo = mid
        else:
            hi, hi_min = mid, mw
            if mw < eps:
                break
    return TPlus(hi, tb, dm, hi_min, solves, False, (lo, hi))
