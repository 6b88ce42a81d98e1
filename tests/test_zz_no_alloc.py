"""The no-allocation entry point mag_residual_noalloc against mag_residual,
called through the C ABI: two calls in a row, the second with a smaller
input (the shared scratch array keeps the first call's contents), an input
above the scratch array's capacity (rejected before any launch), and no
growth of the context's workspace."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _residual_pair(mag, ctx, X, t, w):
    lib = ctx.lib
    n, m = X.shape
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")
    wd = torch.from_numpy(np.ascontiguousarray(w)).to("cuda:0")
    r_ref = torch.empty(n, dtype=torch.float64, device="cuda:0")
    r_na = torch.full((n,), np.nan, dtype=torch.float64, device="cuda:0")
    rinf_ref, rinf_na = ctypes.c_double(), ctypes.c_double()
    torch.cuda.synchronize()
    assert lib.mag_residual(ctx.handle, _ptr(Xd), n, m, t, _ptr(wd), _ptr(r_ref), ctypes.byref(rinf_ref)) == 0
    held = ctx.workspace_bytes()
    assert lib.mag_residual_noalloc(ctx.handle, _ptr(Xd), n, m, t, _ptr(wd), _ptr(r_na), ctypes.byref(rinf_na)) == 0
    assert ctx.workspace_bytes() == held  # nothing grown
    return r_ref.cpu().numpy(), r_na.cpu().numpy(), rinf_ref.value, rinf_na.value


def _check(X, t, w, r_ref, r_na, rinf_ref, rinf_na):
    # both evaluate 1 - Z w in FP64 in different summation orders: they agree
    # to the rounding bound of an n-term sum, 2 n u (|Z||w| + 1)
    n = len(X)
    D = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
    scale = np.exp(-t * D) @ np.abs(w) + 1.0
    tol = 4 * n * U64 * scale
    assert np.all(np.isfinite(r_na))
    assert np.all(np.abs(r_na - r_ref) <= tol)
    assert abs(rinf_na - np.abs(r_na).max()) == 0.0
    assert abs(rinf_na - rinf_ref) <= tol.max()


def test_noalloc_residual_two_calls_then_smaller(mag):
    ctx = mag.Context(0)
    rng = np.random.default_rng(3)
    # first a larger input (several row blocks, column splits and a ragged tail),
    # then a smaller one that leaves the first call's values in the scratch array
    for n, m, t in ((2900, 3, 4.0), (700, 5, 1.5)):
        X = W.gaussian(n, m, seed=n)
        w = rng.standard_normal(n)
        r_ref, r_na, a, b = _residual_pair(mag, ctx, X, t, w)
        _check(X, t, w, r_ref, r_na, a, b)
    ctx.close()


def test_noalloc_residual_high_dimension_and_weighting(mag):
    ctx = mag.Context(0)
    X = W.gaussian(1100, 20, seed=2)
    t = 0.8
    w = mag.weighting(torch.from_numpy(X).to("cuda:0"), t, ctx=ctx).w.cpu().numpy()
    r_ref, r_na, a, b = _residual_pair(mag, ctx, X, t, w)
    _check(X, t, w, r_ref, r_na, a, b)
    assert b <= 1e-12
    ctx.close()


def test_noalloc_rejects_sizes_beyond_scratch(mag):
    ctx = mag.Context(0)
    lib = ctx.lib
    cap = lib.mag_residual_noalloc_max_doubles()
    assert cap == 1 << 21
    n = 1 << 20  # needs 2 npad + npad/256 + 8 > 2^21 doubles
    X = torch.zeros((8, 3), dtype=torch.float64, device="cuda:0")  # never read: rejected first
    w = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    r = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    assert lib.mag_residual_noalloc(ctx.handle, _ptr(X), n, 3, 1.0, _ptr(w), _ptr(r), None) == -4
    assert lib.mag_residual_noalloc(ctx.handle, _ptr(X), 8, 3, -1.0, _ptr(w), _ptr(r), None) == -1
    ctx.close()
