"""The FP64 MFMA blocked Cholesky (solver fp64_chol): the factor, its
diagonal-block inverses and the sync-free FP64 substitution, against the
oracle and against rounding bounds that hold for any correct FP64 Cholesky.

Factor.  A computed Cholesky factor satisfies L L^T = Z + E with
|E| <= gamma_{n+1} |L| |L^T| (Higham, Accuracy and Stability of Numerical
Algorithms, Thm. 10.3), whatever the order of its sums; every row of L has
norm sqrt(Z_jj) = 1, so |L| |L^T| <= 1 entrywise and ||L L^T - Z||_max is
below about (n + 1) u, plus the n u of forming L L^T in numpy.  The sizes
cover the 64-column diagonal blocks, the 128-row tiles and the 256-column
panels on both sides of their edges.

Substitution.  z = (L L^T)^{-1} r against the oracle's residual r - Z z to
1e-12 relative, and the weighting through mag_weighting against the oracle
as for the other solvers.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
SIZES = [2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 767, 1025, 1300]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def colmajor(T):
    """The library's column-major npad x npad buffer as an array A[i, j]."""
    return T.cpu().numpy().T


@pytest.mark.parametrize("n", SIZES)
def test_factor64_backward_error_and_layout(mag, n):
    X = W.gaussian(n, 3, seed=100 + n)
    t = float(W.gaussian_cutoff_estimate(n, 3))
    Lt, dinv_t, bd = mag.factor64(dev(X), t)
    assert bd == 0
    A = colmajor(Lt)
    npad = A.shape[0]
    assert npad == mag.padded_size(n)
    L = np.tril(A[:n, :n])
    Z = oracle.zmatrix(X, t)
    err = float(np.abs(L @ L.T - Z).max())
    bound = 2.0 * (n + 2) * U64
    print(f"n={n} t={t:.4g}: ||L L^T - Z||_max = {err:.3e} (bound {bound:.2e})")
    assert err <= bound
    assert np.all(np.diag(L) > 0)
    # the same factor as the oracle's (unique for an SPD matrix), to its conditioning
    Lo = oracle.cholesky(Z)
    assert float(np.abs(L - Lo).max()) <= 1e-10
    # L^T in the upper triangle, bit for bit
    assert np.array_equal(np.triu(A, 1), np.tril(A, -1).T)
    # identity padding
    if npad > n:
        assert np.array_equal(A[n:, n:], np.eye(npad - n))
        assert not np.any(A[n:, :n]) and not np.any(A[:n, n:])
    # the diagonal-block inverses: lower triangular, inv(L_bb) L_bb = I
    D = dinv_t.cpu().numpy().transpose(0, 2, 1)  # D[b][i, j]
    assert D.shape == (npad // 64, 64, 64)
    for b in range(npad // 64):
        Lb = np.tril(A[64 * b:64 * b + 64, 64 * b:64 * b + 64])
        assert not np.any(np.triu(D[b], 1))
        e = float(np.abs(D[b] @ Lb - np.eye(64)).max())
        kb = np.linalg.cond(Lb)
        assert e <= 64 * 8 * U64 * kb, (b, e, kb)


@pytest.mark.parametrize("n", [65, 257, 700, 1300])
def test_chol64_solve_vs_oracle(mag, n):
    X = W.gaussian(n, 3, seed=200 + n)
    t = float(W.gaussian_cutoff_estimate(n, 3))
    Lt, dinv_t, bd = mag.factor64(dev(X), t)
    assert bd == 0
    r = np.random.default_rng(n).standard_normal(n)
    z = mag.chol64_solve(Lt, dinv_t, n, dev(r)).cpu().numpy()
    res = oracle.residual(X, t, z, b=r)
    rel = float(np.abs(res).max() / np.abs(r).max())
    print(f"n={n}: ||r - Z z||_inf / ||r||_inf = {rel:.3e}")
    assert rel <= 1e-12


def test_fp64_chol_two_points_closed_form(mag):
    # two points at distance d: w_j = 1 / (1 + e^{-t d}) (Section 2)
    X = np.array([[0.0, 0.0], [0.3, 0.4]])
    t = 1.7
    res = mag.weighting(dev(X), t, solver="fp64_chol")
    w = res.w.cpu().numpy()
    ref = 1.0 / (1.0 + np.exp(-t * 0.5))
    assert np.abs(w - ref).max() <= 4 * U64
    assert res.info["solver"] == mag.SOLVERS["fp64_chol"]


def test_fp64_chol_duplicates_rejected(mag):
    X = W.gaussian(300, 3, seed=5)
    X[17] = X[200]
    with pytest.raises(mag.MagError) as e:
        mag.weighting(dev(X), 2.0, solver="fp64_chol")
    assert e.value.code == -2  # MAG_ENOTPD


def test_fp64_chol_matches_vendor_comparator(mag):
    # this library's FP64 factor and rocSOLVER's reach the same weighting
    X = W.gaussian_mixture(1500, 3, seed=4)
    t = 30.0
    a = mag.weighting(dev(X), t, solver="fp64_chol", profile=True)
    b = mag.weighting(dev(X), t, solver="fp64_dense")
    wa, wb = a.w.cpu().numpy(), b.w.cpu().numpy()
    ra = np.abs(oracle.residual(X, t, wa)).max()
    rb = np.abs(oracle.residual(X, t, wb)).max()
    ref = oracle.weighting(X, t)
    _, lmin, _ = oracle.cond_estimate(ref, iters=200, rtol=1e-8)
    bound = 2.0 * np.sqrt(len(X)) * (ra + rb) / lmin
    print(f"fp64_chol resid {ra:.2e}, fp64_dense resid {rb:.2e}, |wa - wb| {np.abs(wa - wb).max():.2e} "
          f"(bound {bound:.2e}); factor {a.info['ms_factor']:.2f} ms")
    assert ra <= 1e-12 and rb <= 1e-12
    assert np.abs(wa - wb).max() <= max(bound, 1e-12 * np.abs(wb).max())
