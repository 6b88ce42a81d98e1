"""Kernel-level parity of the HIP path against the CPU oracle (through the C ABI).

Sizes span several 128/256 tiles and a ragged tail; every input is seeded.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("n,m,seed", [(2, 3, 0), (300, 2, 1), (700, 3, 2), (1025, 8, 3), (513, 11, 4)])
def test_dmin_matches_oracle_bitwise(mag, n, m, seed):
    X = W.gaussian(n, m, seed=seed)
    d_gpu = mag.dmin(dev(X))
    d_orc = oracle.dmin(X)
    # same exact-difference, uncontracted squared sum, same sqrt: identical bits
    assert d_gpu == d_orc


def test_dmin_lattice(mag):
    X = W.z2_rectangles(1500, seed=3)
    assert mag.dmin(dev(X)) == 1.0


@pytest.mark.parametrize("n,m,t", [(200, 3, 2.5), (700, 2, 0.7), (513, 8, 1.0), (300, 12, 0.4)])
def test_tilegen32_matches_oracle(mag, n, m, t):
    X = W.gaussian(n, m, seed=n)
    A = mag.tile32(dev(X), t).cpu().numpy()  # A[j, i] = Z_ij
    npad = A.shape[0]
    Z = oracle.zmatrix(X, t)
    lower = np.tril(np.ones((n, n), dtype=bool))
    got = A[:n, :n].T  # got[i, j] = Z_ij for i >= j (lower triangle written)
    ref = Z.astype(np.float32).astype(np.float64)
    diff = np.abs(got.astype(np.float64) - Z)[lower]
    # FP32 from FP64 differences: x = fl(fl(t) * sqrtf(fl(d^2))) carries up to 3.5
    # unit roundoffs, so |dZ| <= 3.5 U32 x Z, plus expf's own few units
    D = oracle.distance_matrix(X)
    tol = (4 + 4 * t * D) * U32 * Z + 1e-45
    assert np.all(diff <= tol[lower])
    assert np.all(np.diag(got) == 1.0)
    # identity padding
    if npad > n:
        pad = A[n:, :].T  # rows >= n (as Z rows), all columns
        assert np.all(np.diag(A)[n:] == 1.0)
        low = np.tril(np.ones((npad, npad), dtype=bool), -1)
        full = A.T
        assert np.all(full[n:, :][low[n:, :]] == 0.0)
    del ref


@pytest.mark.parametrize("n,m,t", [(1, 3, 1.0), (255, 3, 5.0), (700, 3, 0.8), (2049, 2, 3.0), (600, 8, 1.0), (400, 10, 0.5)])
def test_zmatvec_matches_oracle(mag, n, m, t):
    X = W.gaussian(n, m, seed=7 + n)
    v = np.random.default_rng(n).standard_normal(n)
    y = mag.zmatvec(dev(X), t, dev(v)).cpu().numpy()
    y_ref = oracle.zmatvec(X, t, v)
    scale = oracle.zmatvec(X, t, np.abs(v))
    assert np.all(np.abs(y - y_ref) <= 64 * U64 * scale + 1e-300)


@pytest.mark.parametrize("m,t", [(1, 1.0), (3, 20.0), (10, 5.0)])
def test_zmatvec_entries(mag, m, t):
    # Z e_k is column k of Z, each entry a single product: every FP64 entry
    # exp(-t d_jk) (symmetric product for m <= 8, row product beyond) within 2 ulp
    # of the oracle's libm value, over t d up to 800 (underflow to 0 past ~745)
    n = 2048
    if m == 1:
        X = (np.arange(n, dtype=np.float64) * (800.0 / (n - 1)))[:, None]
    else:
        X = W.gaussian(n, m, seed=31 + m)
    Z = oracle.zmatrix(X, t)
    for k in (0, n // 2 + 1):
        e = np.zeros(n)
        e[k] = 1.0
        y = mag.zmatvec(dev(X), t, dev(e)).cpu().numpy()
        ref = Z[:, k]
        normal = ref >= np.finfo(np.float64).tiny
        assert np.all(np.abs(y[normal] - ref[normal]) <= 2 * 2.0 ** -52 * ref[normal])
        assert np.all(np.abs(y[~normal] - ref[~normal]) <= 1e-322)


@pytest.mark.parametrize("n,m,t", [(300, 3, 4.0), (1000, 3, 1.5)])
def test_residual_matches_oracle(mag, n, m, t):
    X = W.gaussian(n, m, seed=n)
    s = oracle.weighting(X, t)
    w = s.w + 1e-9 * np.random.default_rng(1).standard_normal(n)  # nonzero residual
    r, rinf = mag.residual(dev(X), t, dev(w))
    r = r.cpu().numpy()
    r_ref = oracle.residual(X, t, w)
    scale = oracle.zmatvec(X, t, np.abs(w))
    assert np.all(np.abs(r - r_ref) <= 64 * U64 * scale)
    assert rinf == np.abs(r).max()


@pytest.mark.parametrize("n,m,t", [(256, 3, 3.0), (700, 3, 2.0), (1300, 2, 5.0), (1024, 8, 1.0)])
def test_factor32(mag, n, m, t):
    X = W.gaussian(n, m, seed=3 * n)
    L, dinv, bd = mag.factor32(dev(X), t)
    assert bd == 0
    Lc = L.cpu().numpy().T  # Lc[i, j] = L_ij
    npad = Lc.shape[0]
    Lf = np.tril(Lc).astype(np.float64)
    # the upper triangle holds L^T (written by the factorisation for the backward solve)
    assert np.array_equal(np.triu(Lc, 1), np.tril(Lc, -1).T)
    Z = np.eye(npad)
    Z[:n, :n] = oracle.zmatrix(X, t)
    E = Lf @ Lf.T - Z
    rel = np.linalg.norm(E) / np.linalg.norm(Z)
    assert rel <= 4 * npad * U32, rel
    # factor agrees with LAPACK's FP64 factor of the same Z to FP32 accuracy times cond
    Lref = np.linalg.cholesky(Z)
    ev = np.linalg.eigvalsh(Z[:n, :n])
    cond = ev[-1] / ev[0]
    assert np.abs(Lf - Lref).max() <= 50 * npad * U32 * np.sqrt(cond)
    # identity padding of the factor
    if npad > n:
        assert np.allclose(Lf[n:, n:], np.eye(npad - n), atol=0)
        assert np.all(Lf[n:, :n] == 0)
    # diagonal-block inverses
    D = dinv.cpu().numpy()
    for b in range(npad // 128):
        blk = Lf[128 * b:128 * (b + 1), 128 * b:128 * (b + 1)]
        Db = D[b].T.astype(np.float64)  # column-major 128 x 128
        assert np.abs(Db @ blk - np.eye(128)).max() <= 2e-4


def test_factor32_breakdown_reported(mag):
    # at tiny t, Z is numerically singular in FP32 (Z ~ 1 1^T - t d)
    X = W.gaussian(400, 3, seed=8)
    L, dinv, bd = mag.factor32(dev(X), 1e-7)
    assert bd > 0
    # a large enough diagonal shift restores an FP32 factor
    L, dinv, bd = mag.factor32(dev(X), 1e-7, shift=1e-2)
    assert bd == 0


@pytest.mark.parametrize("n,m,t", [(256, 3, 3.0), (700, 3, 2.0), (2000, 2, 4.0)])
def test_prec_apply(mag, n, m, t):
    X = W.gaussian(n, m, seed=n + 1)
    L, dinv, bd = mag.factor32(dev(X), t)
    assert bd == 0
    Lf = np.tril(L.cpu().numpy().T).astype(np.float64)[:n, :n]
    r = np.random.default_rng(2).standard_normal(n)
    z = mag.prec_apply(L, dinv, n, dev(r)).cpu().numpy()
    z_ref = np.linalg.solve(Lf.T, np.linalg.solve(Lf, r))
    # diagonal blocks applied through FP32 explicit inverses: FP32-level agreement
    assert np.abs(z - z_ref).max() <= 1e-4 * np.abs(z_ref).max()
    # deterministic linear operator: repeat is bitwise identical, and linear
    z2 = mag.prec_apply(L, dinv, n, dev(r)).cpu().numpy()
    assert np.array_equal(z, z2)
    r2 = np.random.default_rng(3).standard_normal(n)
    za = mag.prec_apply(L, dinv, n, dev(r + 2 * r2)).cpu().numpy()
    zb = mag.prec_apply(L, dinv, n, dev(r2)).cpu().numpy()
    assert np.allclose(za, z + 2 * zb, rtol=1e-12, atol=1e-12 * np.abs(za).max())
