"""GPU parity of the weighting at scale zero (mag_weighting_zero, eq. scaleZero:
w0 = d^{-1} 1 / (1^T d^{-1} 1)) against closed forms and the CPU oracle (LU
with partial pivoting on d, Dot2 refinement).

The primary check is the oracle's Dot2 residual of the returned w0: d w0 must
be the constant c* 1 with c* = 1 / (1^T d^{-1} 1).  The solve stops at
||1 - B u||_inf <= 1e-12 for B = c 1 1^T - d, which leaves d w0 - c* 1 = r / beta
(beta = 1^T u), i.e. a relative deviation ||r|| / (c / c* - 1) with c of the
order of a few c*, so 1e-10 relative to c* has margin.  Elementwise agreement
with the oracle is looser: both solutions carry errors up to cond(d) times
their residuals, and cond(d) reaches 1e7 on these sets."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def check_residual(X, w0, sum_dinv, rows=None, tol=1e-10):
    cstar = 1.0 / sum_dinv
    r = oracle.dist_residual(X, w0 / cstar, rows)  # 1 - d (w0 / c*) = (c* 1 - d w0) / c*
    assert np.abs(r).max() <= tol, np.abs(r).max()
    return float(np.abs(r).max())


def test_tiny_cases(mag):
    r = mag.weighting_zero(dev(np.array([[1.0, 2.0]])))
    assert r.w.cpu().numpy().tolist() == [1.0] and r.info["sum_dinv"] == float("inf")
    X = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    r = mag.weighting_zero(dev(X))
    assert np.abs(r.w.cpu().numpy() - 0.5).max() <= 1e-14
    assert r.info["sum_dinv"] == pytest.approx(2.0 / 3.0, rel=1e-13)


@pytest.mark.parametrize("n,m", [(300, 3), (1000, 2)])
def test_collinear_closed_form(mag, n, m):
    X = W.collinear(n, m, seed=n)
    proj = X @ (X[1] - X[0])
    lo, hi = int(np.argmin(proj)), int(np.argmax(proj))
    L = float(np.linalg.norm(X[hi] - X[lo]))
    r = mag.weighting_zero(dev(X))
    w0 = r.w.cpu().numpy()
    ref = np.zeros(n)
    ref[lo] = ref[hi] = 0.5
    print(n, m, r.info, np.abs(w0 - ref).max())
    assert r.info["status"] == 0
    assert np.abs(w0 - ref).max() <= 1e-6
    assert r.info["sum_dinv"] == pytest.approx(2.0 / L, rel=1e-8)
    check_residual(X, w0, r.info["sum_dinv"])


@pytest.mark.parametrize("k", [12, 257])
def test_polygon_closed_form(mag, k):
    X = W.regular_polygon(k)
    rs = sum(2.0 * np.sin(np.pi * l / k) for l in range(1, k))
    r = mag.weighting_zero(dev(X))
    w0 = r.w.cpu().numpy()
    assert np.abs(w0 - 1.0 / k).max() <= 1e-12 / k * 100
    assert r.info["sum_dinv"] == pytest.approx(k / rs, rel=1e-11)


CLOUDS = [
    ("gaussian3", lambda: W.gaussian(1500, 3, seed=0)),
    ("gaussian8", lambda: W.gaussian(1200, 8, seed=1)),
    ("square", lambda: W.uniform_square(2000, seed=2)),
    ("mixture", lambda: W.gaussian_mixture(1700, 3, seed=4)),
    ("torus", lambda: W.noisy_torus(2500, seed=0)),
    ("ragged", lambda: W.gaussian(777, 5, seed=6)),
]


@pytest.mark.parametrize("name,make", CLOUDS, ids=[c[0] for c in CLOUDS])
def test_vs_oracle(mag, name, make):
    X = make()
    r = mag.weighting_zero(dev(X))
    w0 = r.w.cpu().numpy()
    ref, s = oracle.weighting_zero(X)
    res = check_residual(X, w0, r.info["sum_dinv"])
    err = np.abs(w0 - ref).max() / np.abs(ref).max()
    print(name, len(X), r.info["outer_iters"], r.info["gmres_iters"], r.info["shifted"], r.info["c"], res, err)
    assert r.info["status"] == 0
    assert r.info["magnitude"] == pytest.approx(1.0, abs=1e-13)
    assert r.info["sum_dinv"] == pytest.approx(s, rel=1e-8)
    assert err <= 1e-6
    assert r.info["argmin_w"] == int(np.argmin(w0))


def test_errors(mag):
    X = W.gaussian(300, 3, seed=3)
    Xd = X.copy()
    Xd[5] = Xd[9]
    with pytest.raises(mag.MagError):
        mag.weighting_zero(dev(Xd))
    with pytest.raises(mag.MagError):
        mag.weighting_zero(dev(W.gaussian(300, 17, seed=3)))
    with pytest.raises(mag.MagError):
        mag.weighting_zero(dev(X), solver="hodlr")


def test_metric_size_sampled_rows(mag):
    """n = 32768, m = 3 (the metric cloud) at scale zero: the oracle's Dot2
    residual on 256 sampled rows."""
    n, m = 32768, 3
    X = W.gaussian(n, m, seed=0)
    r = mag.weighting_zero(dev(X))
    w0 = r.w.cpu().numpy()
    rows = np.random.default_rng(11).choice(n, size=256, replace=False)
    res = check_residual(X, w0, r.info["sum_dinv"], rows)
    print(r.info, res)
    assert r.info["status"] == 0
