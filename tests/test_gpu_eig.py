"""GPU parity of the extreme-eigenvalue estimator (mag_eig_extremes, the
positive-definiteness check of Section 4.2) against closed forms, the
eigenvalues numpy's eigvalsh gives for the oracle's FP64 Z, and properties
that hold at any size.

Lanczos bounds used by the checks: the Ritz value theta of the top side of an
operator with eigenvalues mu_1 > mu_2 >= ... satisfies theta <= mu_1 (Cauchy
interlacing), and with residual bound r and theta > mu_2, mu_1 - theta <=
r^2 / (theta - mu_2) (Kato-Temple).  The lambda_min side is the top side of
Z^{-1} (mu = 1/lambda).  A slack of 1e-10 relative covers FP64 rounding of the
products and the 1e-12 tolerance of each inner solve."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

SLACK = 1e-10


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def check_top(theta, r, mu1, mu2, converged, what):
    """theta: Ritz value of the top side; mu1 > mu2 the operator's two largest
    distinct eigenvalues."""
    assert theta <= mu1 * (1 + SLACK), (what, theta, mu1)
    if converged and theta > mu2:
        bound = r * r / (theta - mu2)
        assert mu1 - theta <= bound + SLACK * mu1, (what, theta, mu1, r, bound)


def polygon_spectrum(k, t):
    """Eigenvalues of Z for the regular k-gon of unit circumradius: Z is
    circulant with first row f_l = exp(-2 t sin(pi l / k)), so its eigenvalues
    are the real DFT values sum_l f_l cos(2 pi p l / k), p = 0..k-1."""
    l = np.arange(k)
    f = np.exp(-2.0 * t * np.sin(np.pi * l / k))
    p = l[:, None]
    return np.sort((f[None, :] * np.cos(2.0 * np.pi * p * l[None, :] / k)).sum(axis=1))


def distinct_top2(vals, rel=1e-9):
    """The largest value and the largest one below it by more than rel."""
    v = np.sort(vals)[::-1]
    mu1 = v[0]
    rest = v[v < mu1 * (1 - rel)]
    return mu1, (rest[0] if rest.size else -np.inf)


def check_against_spectrum(info, lam, what):
    lam = np.sort(lam)
    mu1, mu2 = distinct_top2(lam)
    check_top(info["lambda_max"], info["resid_max"], mu1, mu2, info["converged"] & 1, what + " max")
    inv = 1.0 / lam
    nu1, nu2 = distinct_top2(inv)
    check_top(1.0 / info["lambda_min"], info["resid_min"], nu1, nu2, info["converged"] & 2, what + " min")


def test_one_and_two_points(mag):
    info = mag.eig_extremes(dev(np.array([[0.3, -1.0, 2.0]])), 5.0)
    assert info["status"] == 0 and info["lambda_max"] == pytest.approx(1.0, abs=1e-15)
    assert info["lambda_min"] == pytest.approx(1.0, abs=1e-13) and info["converged"] == 3
    # two points at distance d: Z = [[1, q], [q, 1]], q = exp(-t d), eigenvalues 1 +- q
    d, t = 0.75, 1.3
    X = np.array([[0.0, 0.0], [d, 0.0]])
    info = mag.eig_extremes(dev(X), t)
    q = np.exp(-t * d)
    assert info["converged"] == 3 and info["iters_max"] <= 2 and info["iters_min"] <= 2
    assert abs(info["lambda_max"] - (1 + q)) <= 1e-14
    assert abs(info["lambda_min"] - (1 - q)) <= 1e-12
    assert info["cond"] == pytest.approx((1 + q) / (1 - q), rel=1e-12)


@pytest.mark.parametrize("k,t", [(64, 1.0), (257, 0.5), (1000, 2.0)])
def test_regular_polygon_closed_form(mag, k, t):
    lam = polygon_spectrum(k, t)
    info = mag.eig_extremes(dev(W.regular_polygon(k)), t, max_iter=120)
    print(k, t, info, lam[0], lam[-1])
    assert info["status"] == 0
    check_against_spectrum(info, lam, f"k-gon {k}")
    # lambda_max is well separated here: converged to rtol
    assert info["converged"] & 1
    assert abs(info["lambda_max"] - lam[-1]) <= 1e-12 * lam[-1]


@pytest.mark.parametrize("n,m,tfac,seed", [(700, 3, 1.0, 0), (1500, 3, 0.25, 1), (2100, 8, 1.0, 2),
                                           (1024, 2, 4.0, 3)])
def test_vs_eigvalsh(mag, n, m, tfac, seed):
    X = W.gaussian(n, m, seed=seed)
    t = tfac * float(W.gaussian_cutoff_estimate(n, m))
    lam = np.linalg.eigvalsh(oracle.zmatrix(X, t))
    info = mag.eig_extremes(dev(X), t, max_iter=200)
    print(n, m, t, info, lam[0], lam[-1])
    assert info["status"] == 0
    check_against_spectrum(info, lam, f"gaussian {n}x{m}")
    assert info["converged"] & 1
    assert abs(info["lambda_max"] - lam[-1]) <= 1e-10 * lam[-1]
    if info["converged"] & 2:
        assert abs(info["lambda_min"] - lam[0]) <= 1e-6 * lam[0]


def test_caller_start_vector_and_errors(mag):
    X = W.gaussian(600, 3, seed=4)
    t = 4.0
    lam = np.linalg.eigvalsh(oracle.zmatrix(X, t))
    v0 = np.random.default_rng(5).standard_normal(600)
    info = mag.eig_extremes(dev(X), t, v0=dev(v0), max_iter=150)
    check_against_spectrum(info, lam, "v0")
    with pytest.raises(mag.MagError):
        mag.eig_extremes(dev(X), t, v0=dev(np.zeros(600)))
    Xd = X.copy()
    Xd[7] = Xd[3]
    with pytest.raises(mag.MagError):
        mag.eig_extremes(dev(Xd), t)
    with pytest.raises(mag.MagError):
        mag.eig_extremes(dev(X), t, max_iter=300)
    with pytest.raises(mag.MagError):
        mag.eig_extremes(dev(X), t, solver="hodlr")


def test_metric_workload_properties(mag):
    """n = 32768, m = 3 at the Gaussian cutoff scale: no eigendecomposition is
    possible here, so properties that hold at any size: the diagonal of Z is 1,
    so lambda_min <= 1 <= lambda_max; lambda_max >= the Rayleigh quotient of
    the ones vector (1^T Z 1 / n, the oracle's row sums); Mag = 1^T Z^{-1} 1
    lies in [n / lambda_max, n / lambda_min]; Z is positive definite."""
    n, m = 32768, 3
    X = W.gaussian(n, m, seed=0)
    t = float(W.gaussian_cutoff_estimate(n, m))
    Xd = dev(X)
    info = mag.eig_extremes(Xd, t)
    M = mag.weighting(Xd, t, solver="fp32_ir").info["magnitude"]
    rows = np.arange(n)
    ones = np.ones(n)
    rayleigh = float((1.0 - oracle.residual(X, t, ones, rows)).sum()) / n
    print(info, rayleigh, M)
    assert info["status"] == 0 and info["converged"] & 1
    assert 0.0 < info["lambda_min"] <= 1.0 <= info["lambda_max"]
    assert info["lambda_max"] >= rayleigh * (1 - SLACK)
    assert n / info["lambda_max"] * (1 - 1e-9) <= M <= n / info["lambda_min"] * (1 + 1e-9)
