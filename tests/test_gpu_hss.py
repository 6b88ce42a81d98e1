"""HSS-preconditioned solves (MAG_HSS: nested bases, ULV factor) against the
CPU oracle and closed forms.

As for the HODLR, the factor itself (tree, bases, ranks) is not unique, so the
final weighting is what is compared: ||1 - Z w||_inf <= 1e-12 with the oracle's
Dot2 residual, and the magnitude where kappa_M allows.  Two cases pin the
factorisation itself:
  * collinear points: every off-diagonal block row of exp(-t |x - y|) on a
    line has rank 2 (exp(-t x) exp(t y) on one side, exp(t x) exp(-t y) on the
    other), so the HSS form with nested bases is exact and the preconditioned
    solve converges in one plain step; the weights then match their closed
    form (tanh of half the scaled gaps);
  * one leaf (n <= leaf): the root block is Z, factored by Cholesky.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from parity_util import w_tolerance

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def check(X, t, res, m_tol=1e-10):
    w = res.w.cpu().numpy()
    ref = oracle.weighting(X, t)
    r = np.abs(oracle.residual(X, t, w)).max()
    assert r <= 1e-12, f"residual {r:.3e}"
    kM = oracle.kappa_M(ref)
    errM = abs(res.info["magnitude"] - ref.M) / abs(ref.M)
    if 2 * U64 * kM <= 1e-11:
        assert errM <= m_tol, f"M rel err {errM:.3e} (kappa_M {kM:.3e})"
    else:
        assert errM <= 8 * U64 * kM + m_tol
    assert res.info["argmin_w"] == int(np.argmin(w))
    return w, ref, errM


@pytest.mark.parametrize("n,t", [(1000, 3.0), (3000, 0.7)])
def test_hss_collinear_exact(mag, n, t):
    X = W.collinear(n, 3, seed=n)
    res = mag.weighting(dev(X), t, solver="hss")
    w = res.w.cpu().numpy()
    # closed form on a line: ends (1 + tanh(t g / 2)) / 2, interior (tanh(t g_-/2) + tanh(t g_+/2)) / 2
    proj = X @ (X[1] - X[0])
    order = np.argsort(proj)
    g = np.linalg.norm(np.diff(X[order], axis=0), axis=1)
    th = np.tanh(t * g / 2)
    ref = np.empty(n)
    ref[order[0]] = (1 + th[0]) / 2
    ref[order[-1]] = (1 + th[-1]) / 2
    ref[order[1:-1]] = (th[:-1] + th[1:]) / 2
    # the solve stops at ||1 - Z w||_inf <= 1e-12, so |w - w_exact| <= ||Z^{-1}||_inf 1e-12
    bound = 1e-12 * np.abs(np.linalg.inv(oracle.zmatrix(X, t))).sum(axis=1).max()
    print(n, t, res.info["outer_iters"], res.info["gmres_iters"], np.abs(w - ref).max(), bound)
    assert np.abs(w - ref).max() <= 2 * bound + 1e-14
    assert res.info["gmres_iters"] <= 2  # an exact preconditioner: the plain steps converge


CASES = [
    ("single_leaf100", lambda: W.gaussian(100, 3, seed=15), 2.0, {}),
    ("two_leaves200", lambda: W.gaussian(200, 3, seed=16), 2.0, {}),
    ("torus2000_t05", lambda: W.noisy_torus(2000, seed=5), 0.5, {}),
    ("torus2000_t8", lambda: W.noisy_torus(2000, seed=5), 8.0, {}),
    ("gauss3001_tstar", lambda: W.gaussian(3001, 3, seed=11), W.gaussian_cutoff_estimate(3001, 3), {}),
    ("gauss1200_m8_t1", lambda: W.gaussian(1200, 8, seed=12), 1.0, {}),
    ("mixture2500_t30", lambda: W.gaussian_mixture(2500, 3, seed=14), 30.0, {}),
    ("square4000_rank512", lambda: W.uniform_square(4000, seed=3), 20.0, {"max_rank": 512}),
    ("torus5000_rank64", lambda: W.noisy_torus(5000, seed=7), 2.0, {"max_rank": 64, "oversample": 0,
                                                                     "gmres_restart": 100, "max_gmres": 400}),
    ("torus5000_leaf256_rank64", lambda: W.noisy_torus(5000, seed=7), 2.0,
     {"leaf": 256, "max_rank": 64, "oversample": 0, "gmres_restart": 100, "max_gmres": 400}),
    ("gauss3001_leaf256_tstar", lambda: W.gaussian(3001, 3, seed=11), W.gaussian_cutoff_estimate(3001, 3),
     {"leaf": 256}),
    ("gauss2000_m16_leaf256_t1", lambda: W.gaussian(2000, 16, seed=20), 1.0, {"leaf": 256}),
]


@pytest.mark.parametrize("name,mkX,t,kw", CASES, ids=[c[0] for c in CASES])
def test_hss_parity(mag, name, mkX, t, kw):
    X = mkX()
    res = mag.weighting(dev(X), float(t), solver="hss", **kw)
    w, ref, errM = check(X, float(t), res)
    tol_w, _ = w_tolerance(X, float(t), w, ref)
    relw = np.abs(w - ref.w).max() / np.abs(ref.w).max()
    assert np.abs(w - ref.w).max() <= tol_w
    hod = mag.weighting(dev(X), float(t), solver="hodlr", **kw).info
    print(f"{name}: n={len(X)} t={t:.4g} relerr_w={relw:.2e} relerr_M={errM:.2e} "
          f"outer={res.info['outer_iters']} gmres={res.info['gmres_iters']} (hodlr gmres={hod['gmres_iters']})")


def test_hss_deterministic_and_errors(mag):
    X = W.noisy_torus(1500, seed=3)
    a = mag.weighting(dev(X), 1.0, solver="hss").w.cpu().numpy()
    b = mag.weighting(dev(X), 1.0, solver="hss").w.cpu().numpy()
    assert np.array_equal(a, b)
    with pytest.raises(mag.MagError):  # leaves below 64 points
        mag.weighting(dev(X), 1.0, solver="hss", leaf=32)
    with pytest.raises(mag.MagError):
        mag.weighting(dev(W.gaussian(300, 17, seed=1)), 1.0, solver="hss")
    Xd = W.gaussian(400, 3, seed=2)
    Xd[7] = Xd[300]
    with pytest.raises(mag.MagError):
        mag.weighting(dev(Xd), 1.0, solver="hss")
