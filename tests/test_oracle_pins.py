"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with a
closed form, an invariant, an independent library routine (SciPy / numpy
LAPACK, which the oracle does not call), exact rational arithmetic, or a
value the paper prints.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import scipy.spatial.distance

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- closed forms

def test_single_point():
    X = np.array([[0.3, -1.2, 4.0]])
    s = oracle.weighting(X, 2.5)
    assert s.w.tolist() == [1.0]
    assert s.M == 1.0


@pytest.mark.parametrize("t", [1e-3, 0.3, 1.0, 7.0, 40.0])
def test_two_points(t):
    # Z = [[1, q], [q, 1]], q = exp(-t d): w_j = 1/(1+q), M = 1 + tanh(t d / 2).
    X = np.array([[0.0, 0.0], [0.6, 0.8]])  # d = 1
    d = 1.0
    s = oracle.weighting(X, t)
    wexp = 1.0 / (1.0 + np.exp(-t * d))
    assert np.allclose(s.w, wexp, rtol=1e-14, atol=0)
    assert abs(s.M - (1.0 + np.tanh(t * d / 2))) <= 1e-14 * s.M


@pytest.mark.parametrize("n,m,t", [(7, 3, 0.5), (40, 2, 2.0), (200, 5, 0.05), (64, 1, 30.0)])
def test_collinear_closed_form(n, m, t):
    # Z^{-1} is tridiagonal for points on a line (Ornstein-Uhlenbeck kernel):
    # endpoint weights (1 + tanh(t g/2))/2, interior (tanh(t g_{j-1}/2) + tanh(t g_j/2))/2,
    # M = 1 + sum_i tanh(t g_i / 2).
    X = W.collinear(n, m, seed=n)
    s_pos = np.linalg.norm(X - X[0], axis=1)
    order = np.argsort(s_pos)
    g = np.diff(s_pos[order])
    th = np.tanh(t * g / 2)
    wexp = np.empty(n)
    wexp[0] = (1 + th[0]) / 2
    wexp[-1] = (1 + th[-1]) / 2
    wexp[1:-1] = (th[:-1] + th[1:]) / 2
    sol = oracle.weighting(X, t)
    w_sorted = sol.w[order]
    cond_scale = max(1.0, 1.0 / (t * g.min()))
    assert np.allclose(w_sorted, wexp, rtol=0, atol=1e-13 * cond_scale)
    assert abs(sol.M - (1 + th.sum())) <= 1e-13 * cond_scale * n


@pytest.mark.parametrize("t,delta", [(0.01, 0.2), (0.7, 0.05), (3.0, 0.5), (10.0, 1e-3), (25.0, 1.3)])
def test_example1_closed_form(t, delta):
    # Section 2, Example 1: d12 = d13 = 1, d23 = delta; realise it in R^2.
    a = np.arcsin(delta / 2)
    X = np.array([[0.0, 0.0], [np.cos(a), np.sin(a)], [np.cos(a), -np.sin(a)]])
    den = np.exp((delta + 2) * t) - 2 * np.exp(delta * t) + np.exp(2 * t)
    w1 = (np.exp((delta + 2) * t) - 2 * np.exp((delta + 1) * t) + np.exp(2 * t)) / den
    w2 = (np.exp((delta + 2) * t) - np.exp((delta + 1) * t)) / den
    s = oracle.weighting(X, t)
    scale = max(1.0, 1.0 / (t * delta))  # cond grows as delta t -> 0
    assert np.allclose(s.w, [w1, w2, w2], rtol=1e-12 * scale, atol=1e-12 * scale)


def test_example1_printed_limits():
    spec = json.load(open(os.path.join(GOLD, "example1_limits.json")))
    delta = spec["delta"]
    a = np.arcsin(delta / 2)
    X = np.array([[0.0, 0.0], [np.cos(a), np.sin(a)], [np.cos(a), -np.sin(a)]])
    for c in spec["cases"]:
        s = oracle.weighting(X, c["t"])
        assert np.allclose(s.w, c["w"], atol=c["abs_tol"]), (c, s.w)


def _kgon_root(k):
    # centre + regular k-gon (unit circumradius): w_c = (S - k q)/(S - k q^2) with
    # q = e^{-t}, S = 1 + sum_{j=1}^{k-1} exp(-2 t sin(pi j/k)); t_+ solves S = k e^{-t}.
    def f(t):
        S = 1 + sum(np.exp(-2 * t * np.sin(np.pi * j / k)) for j in range(1, k))
        return S - k * np.exp(-t)
    return scipy.optimize.brentq(f, 0.05, 10.0, xtol=1e-15, rtol=1e-15)


@pytest.mark.parametrize("k,t", [(6, 0.5), (8, 1.3), (12, 3.0)])
def test_kgon_weights_closed_form(k, t):
    X = W.centre_kgon(k)
    q = np.exp(-t)
    S = 1 + sum(np.exp(-2 * t * np.sin(np.pi * j / k)) for j in range(1, k))
    wc = (S - k * q) / (S - k * q * q)
    wr = (1 - q) / (S - k * q * q)
    s = oracle.weighting(X, t)
    assert np.allclose(s.w, [wc] + [wr] * k, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("k", [6, 8, 12])
def test_kgon_tplus_pin(k):
    root = _kgon_root(k)
    r = oracle.tplus(W.centre_kgon(k), rtol=1e-7)
    assert not r.no_sign_change
    # returned t_+ is the upper end of a bracket of relative width <= rtol
    assert root <= r.t_plus * (1 + 1e-12)
    assert (r.t_plus - root) / root <= 2e-7
    # brute-force sign checks around the cutoff
    X = W.centre_kgon(k)
    assert oracle.weighting(X, root * (1 + 1e-5)).min_w >= 0
    assert oracle.weighting(X, root * (1 - 1e-5)).min_w < 0


def test_tplus_known_values():
    # values of the k-gon root quoted for calibration (brentq on the closed form)
    assert abs(_kgon_root(6) - 0.96985176877400) < 1e-12
    assert abs(_kgon_root(24) - 1.32829005030313) < 1e-12


# ---------------------------------------------------------------- invariants

def test_large_t_magnitude_tends_to_n():
    X = W.uniform_square(64, seed=3)
    dm = oracle.dmin(X)
    t = 40.0 / dm  # every off-diagonal Z_jk <= e^{-40}
    s = oracle.weighting(X, t)
    assert abs(s.M - 64) < 64 * 64 * np.exp(-40)
    assert s.min_w > 1 - 64 * np.exp(-40)


def test_small_t_limit_scale_zero():
    # eq. scaleZero: w(t) -> d^{-1} 1 / (1^T d^{-1} 1) and M -> 1 as t -> 0, error O(t)
    X = W.uniform_square(12, seed=4, m=3)
    D = scipy.spatial.distance.cdist(X, X)
    w0 = np.linalg.solve(D, np.ones(12))
    w0 = w0 / w0.sum()
    errs = []
    for t in (1e-2, 1e-3):
        s = oracle.weighting(X, t)
        errs.append(np.abs(s.w - w0).max())
        assert abs(s.M - 1) < 10 * t
    assert errs[1] < errs[0] / 5  # O(t) convergence


def test_scaling_homogeneity():
    # w(t; lambda X) = w(lambda t; X); t_+(lambda X) = t_+(X) / lambda (Appendix C.2)
    X = W.gaussian(50, 3, seed=5)
    lam = 3.7
    a = oracle.weighting(lam * X, 0.8).w
    b = oracle.weighting(X, 0.8 * lam).w
    assert np.allclose(a, b, rtol=1e-11, atol=1e-12)
    ta = oracle.tplus(lam * X).t_plus
    tb = oracle.tplus(X).t_plus
    assert abs(ta * lam - tb) / tb < 3e-6


def test_weights_nonnegative_at_bound():
    for seed in range(3):
        X = W.gaussian(80, 2, seed=seed)
        s = oracle.weighting(X, oracle.t_bound(X))
        assert s.min_w >= 0


def test_permutation_rotation_translation():
    X = W.gaussian(60, 3, seed=6)
    t = 1.1
    w = oracle.weighting(X, t).w
    P = np.random.default_rng(1).permutation(60)
    assert np.allclose(oracle.weighting(X[P], t).w, w[P], rtol=1e-12, atol=1e-13)
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((3, 3)))
    Y = X @ Q.T + np.array([5.0, -2.0, 0.25])
    assert np.allclose(oracle.weighting(Y, t).w, w, rtol=1e-10, atol=1e-11)


def test_diversity_identity():
    # q = 2 diversity identity: w^T Z w = 1^T w when Z w = 1 (Section 2)
    X = W.gaussian(100, 3, seed=8)
    t = 0.9
    s = oracle.weighting(X, t)
    Z = scipy.spatial.distance.cdist(X, X)
    Z = np.exp(-t * Z)
    assert abs(s.w @ Z @ s.w - s.w.sum()) < 1e-10 * abs(s.w.sum())


# ---------------------------------------------------------------- library reductions

@pytest.mark.parametrize("n,m,t", [(300, 3, 2.0), (257, 2, 0.3), (129, 8, 1.0)])
def test_vs_scipy_cho_solve(n, m, t):
    X = W.gaussian(n, m, seed=n)
    s = oracle.weighting(X, t)
    Z = np.exp(-t * scipy.spatial.distance.cdist(X, X))
    w_ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(Z, lower=True), np.ones(n))
    lam = np.linalg.eigvalsh(Z)
    cond = lam[-1] / lam[0]
    assert np.allclose(s.w, w_ref, rtol=0, atol=50 * cond * 2.2e-16 * np.abs(w_ref).max())
    assert abs(s.M - w_ref.sum()) <= 50 * cond * 2.2e-16 * np.abs(w_ref).sum()


def test_distance_and_dmin_vs_scipy():
    X = W.gaussian(150, 4, seed=9)
    D = oracle.distance_matrix(X)
    Dref = scipy.spatial.distance.cdist(X, X)
    assert np.allclose(D, Dref, rtol=4e-16, atol=0)
    assert oracle.dmin(X) == pytest.approx(scipy.spatial.distance.pdist(X).min(), rel=4e-16)


def test_zmatrix_vs_numpy():
    X = W.uniform_square(90, seed=10)
    t = 3.3
    Z = oracle.zmatrix(X, t)
    Zref = np.exp(-t * scipy.spatial.distance.cdist(X, X))
    assert np.allclose(Z, Zref, rtol=1e-15, atol=0)
    assert np.all(np.diag(Z) == 1.0)
    assert np.array_equal(Z, Z.T)


def test_cholesky_vs_lapack():
    X = W.gaussian(200, 3, seed=11)
    Z = np.exp(-1.5 * scipy.spatial.distance.cdist(X, X))
    L = oracle.cholesky(Z)
    Lref = np.linalg.cholesky(Z)
    assert np.allclose(L, Lref, rtol=0, atol=1e-13)
    assert np.allclose(L @ L.T, Z, atol=1e-14)


def test_cholesky_detects_non_pd():
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 0.0]])  # duplicate point -> singular Z
    with pytest.raises(oracle.NotPositiveDefinite):
        oracle.weighting(X, 1.0)


def test_chol_solve_vs_lapack():
    rng = np.random.default_rng(12)
    A = rng.standard_normal((60, 60))
    A = A @ A.T + 60 * np.eye(60)
    b = rng.standard_normal(60)
    L = oracle.cholesky(A)
    assert np.allclose(oracle.chol_solve(L, b), np.linalg.solve(A, b), rtol=1e-12, atol=1e-14)


def test_residual_dot2_exact_rational():
    # Dot2 residual vs exact rational arithmetic on the same FP64 Z entries
    X = W.gaussian(40, 3, seed=13)
    t = 0.7
    s = oracle.weighting(X, t, refine=0)
    Z = oracle.zmatrix(X, t)
    r = oracle.residual(X, t, s.w)
    for j in range(40):
        exact = Fraction(1) - sum(Fraction(Z[j, k]) * Fraction(s.w[k]) for k in range(40))
        ex = float(exact)
        bound = 2.0 ** -52 * abs(ex) + 1e-28 * float(sum(abs(Fraction(Z[j, k]) * Fraction(s.w[k])) for k in range(40)))
        assert abs(r[j] - ex) <= bound, (j, r[j], ex)
    # rows subset gives the same numbers
    rows = np.array([3, 0, 39])
    assert np.array_equal(oracle.residual(X, t, s.w, rows), r[rows])


def test_refinement_reaches_unit_roundoff():
    X = W.gaussian(400, 3, seed=14)
    t = W.gaussian_cutoff_estimate(400, 3) / 4  # ill-conditioned side
    s = oracle.weighting(X, t)
    assert np.abs(oracle.residual(X, t, s.w)).max() < 1e-14
    assert np.abs(oracle.residual(X, t, s.w)).max() <= np.abs(oracle.residual(X, t, s.w_plain)).max()


def test_msum_exact():
    rng = np.random.default_rng(15)
    v = rng.standard_normal(1000) * 10.0 ** rng.integers(-8, 8, 1000)
    exact = float(sum(Fraction(x) for x in v))
    assert oracle.msum(v) == pytest.approx(exact, rel=2.3e-16, abs=0)


def test_cond_estimate_vs_eigvalsh():
    X = W.gaussian(300, 3, seed=16)
    t = 2.0
    s = oracle.weighting(X, t)
    lmax, lmin, cond = oracle.cond_estimate(s)
    ev = np.linalg.eigvalsh(oracle.zmatrix(X, t))
    assert lmax == pytest.approx(ev[-1], rel=1e-6)
    assert lmin == pytest.approx(ev[0], rel=1e-4)
    assert cond == pytest.approx(ev[-1] / ev[0], rel=1e-4)


# ---------------------------------------------------------------- gradients

def test_two_point_gradients_closed_form():
    X = np.array([[0.1, 0.2, 0.0], [0.9, -0.3, 0.4]])
    d = float(np.linalg.norm(X[0] - X[1]))
    t = 1.7
    dt, dX, s = oracle.grad(X, t)
    assert dt == pytest.approx(2 * d * np.exp(-t * d) / (1 + np.exp(-t * d)) ** 2, rel=1e-13)
    # M = 1 + tanh(t d / 2): dM/dx_0 = (t/2) sech^2(t d/2) (x_0 - x_1)/d
    g0 = (t / 2) / np.cosh(t * d / 2) ** 2 * (X[0] - X[1]) / d
    assert np.allclose(dX[0], g0, rtol=1e-13)
    assert np.allclose(dX[1], -g0, rtol=1e-13)


def test_collinear_dM_dt_closed_form():
    X = W.collinear(30, 2, seed=3)
    t = 0.9
    s_pos = np.sort(np.linalg.norm(X - X[0], axis=1))
    g = np.diff(s_pos)
    dt, _, _ = oracle.grad(X, t)
    assert dt == pytest.approx(np.sum(g / 2 / np.cosh(t * g / 2) ** 2), rel=1e-11)


def test_gradients_vs_finite_differences():
    rng = np.random.default_rng(17)
    n, m, t = 60, 4, 0.8
    X = W.gaussian(n, m, seed=17)
    gw = rng.standard_normal(n)
    gM = 0.7

    def L(Xv, tv):
        s = oracle.weighting(Xv, tv)
        return gM * s.M + gw @ s.w

    dt, dX, _ = oracle.grad(X, t, gM=gM, gw=gw)
    h = 1e-6
    fd_t = (L(X, t + h) - L(X, t - h)) / (2 * h)
    assert dt == pytest.approx(fd_t, rel=1e-6)
    for _ in range(3):
        V = rng.standard_normal((n, m))
        fd = (L(X + h * V, t) - L(X - h * V, t)) / (2 * h)
        assert float(np.sum(dX * V)) == pytest.approx(fd, rel=1e-6)
    # single coordinates
    for (j, l) in [(0, 0), (17, 3), (59, 1)]:
        E = np.zeros((n, m))
        E[j, l] = 1.0
        fd = (L(X + h * E, t) - L(X - h * E, t)) / (2 * h)
        assert dX[j, l] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_dw_dt_vs_finite_differences():
    X = W.gaussian(50, 3, seed=18)
    t, h = 1.2, 1e-6
    s = oracle.weighting(X, t)
    fd = (oracle.weighting(X, t + h).w - oracle.weighting(X, t - h).w) / (2 * h)
    assert np.allclose(oracle.dw_dt(s), fd, rtol=1e-6, atol=1e-8)


# ---------------------------------------------------------------- cutoff search

def test_collinear_no_sign_change():
    r = oracle.tplus(W.collinear(20, 3, seed=1))
    assert r.no_sign_change and r.t_plus == 0.0


def test_tplus_small_n():
    assert oracle.tplus(np.zeros((1, 2))).no_sign_change
    assert oracle.tplus(np.array([[0.0], [1.0]])).no_sign_change


def test_tplus_brute_force_signs_random_cloud():
    X = W.gaussian_mixture(150, 3, seed=3)
    r = oracle.tplus(X)
    assert not r.no_sign_change
    assert oracle.weighting(X, r.t_plus * (1 + 1e-5)).min_w >= 0
    assert oracle.weighting(X, r.t_plus * (1 - 1e-5)).min_w < 0
    assert r.t_plus <= r.t_bound


def test_gaussian_cutoff_law_loose():
    spec = json.load(open(os.path.join(GOLD, "gaussian_cutoff_law.json")))
    for c in spec["cases"]:
        vals = [oracle.tplus(W.gaussian(c["n"], c["m"], seed=s), rtol=1e-3).t_plus for s in c["seeds"]]
        law = spec["gamma_plus"] * c["m"] ** (-2 / 3) * c["n"] ** 0.25
        assert abs(np.mean(vals) - law) / law < c["rel_tol"], (vals, law)


def test_grad_x_rows_matches_full():
    X = W.gaussian(70, 3, seed=19)
    t = 0.6
    dt, dX, s = oracle.grad(X, t)
    rows = np.array([0, 33, 69])
    got = oracle.grad_x_rows(X, t, s.w, s.w, rows)
    assert np.array_equal(got, dX[rows])


# ---------------------------------------------------------------- scale zero (eq. scaleZero)

def test_scale_zero_tiny_cases():
    w0, s = oracle.weighting_zero(np.array([[0.5, -1.0]]))
    assert w0.tolist() == [1.0] and s == float("inf")
    # two points at distance D: d^{-1} 1 = (1/D, 1/D)
    X = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    w0, s = oracle.weighting_zero(X)
    assert np.allclose(w0, [0.5, 0.5], rtol=0, atol=1e-15) and s == pytest.approx(2.0 / 3.0, rel=1e-15)


@pytest.mark.parametrize("n,m", [(7, 1), (40, 3), (150, 2)])
def test_scale_zero_collinear_closed_form(n, m):
    # on a line, d w = c 1 holds for w = (e_first + e_last) / 2 with c = L / 2, since
    # d_j,first + d_j,last = L for every point j between the ends
    X = W.collinear(n, m, seed=n)
    proj = X @ (X[1] - X[0])
    lo, hi = int(np.argmin(proj)), int(np.argmax(proj))
    L = float(np.linalg.norm(X[hi] - X[lo]))
    w0, s = oracle.weighting_zero(X)
    ref = np.zeros(n)
    ref[lo] = ref[hi] = 0.5
    assert np.abs(w0 - ref).max() <= 1e-10
    assert s == pytest.approx(2.0 / L, rel=1e-10)


@pytest.mark.parametrize("k", [5, 12, 31])
def test_scale_zero_polygon_closed_form(k):
    # regular k-gon: every row of d sums to sum_l 2 sin(pi l / k), so d^{-1} 1 is uniform
    X = W.regular_polygon(k, m=3)
    r = sum(2.0 * np.sin(np.pi * l / k) for l in range(1, k))
    w0, s = oracle.weighting_zero(X)
    assert np.abs(w0 - 1.0 / k).max() <= 1e-14
    assert s == pytest.approx(k / r, rel=1e-13)


@pytest.mark.parametrize("n,m,seed", [(60, 2, 0), (300, 3, 1), (500, 8, 2)])
def test_scale_zero_vs_lapack_and_limit(n, m, seed):
    X = W.gaussian(n, m, seed=seed)
    w0, s = oracle.weighting_zero(X)
    D = scipy.spatial.distance.cdist(X, X)
    u = scipy.linalg.solve(D, np.ones(n))
    assert np.abs(w0 - u / u.sum()).max() <= 1e-9 * np.abs(w0).max()
    assert s == pytest.approx(u.sum(), rel=1e-9)
    # the limit of the finite-scale weighting, with O(t) error
    e1 = np.abs(oracle.weighting(X, 1e-3).w - w0).max()
    e2 = np.abs(oracle.weighting(X, 1e-4).w - w0).max()
    assert e2 < e1 / 5
    # scale invariance of w0; 1^T d^{-1} 1 scales as 1/lambda; permutation equivariance
    w0s, ss = oracle.weighting_zero(2.5 * X)
    assert np.abs(w0s - w0).max() <= 1e-12 * np.abs(w0).max() and ss == pytest.approx(s / 2.5, rel=1e-12)
    perm = np.random.default_rng(seed).permutation(n)
    w0p, _ = oracle.weighting_zero(X[perm])
    assert np.abs(w0p - w0[perm]).max() <= 1e-12 * np.abs(w0).max()


def test_scale_zero_dist_residual_exact_rational():
    # Dot2 residual against exact rationals on a tiny set with integer distances
    X = np.array([[0.0, 0.0], [3.0, 4.0], [6.0, 8.0], [0.0, 5.0]])
    u = np.array([0.1, -0.7, 1.0 / 3.0, 2.5])
    D = [[Fraction(0)] * 4 for _ in range(4)]
    for j in range(4):
        for k in range(4):
            dd = float(np.sqrt(((X[j] - X[k]) ** 2).sum()))
            D[j][k] = Fraction(dd)
    exact = [float(1 - sum(D[j][k] * Fraction(u[k]) for k in range(4))) for j in range(4)]
    assert oracle.dist_residual(X, u).tolist() == exact


# ---------------------------------------------------------------- general right-hand side, kappa_M, LAPACK factor

def test_residual_rhs_dot2_exact_rational():
    # b - Z x by Dot2 vs exact rational arithmetic on the same FP64 entries, for a
    # right-hand side other than 1 (the gradient's lambda = Z^{-1}(gM 1 + gw))
    X = W.gaussian(30, 3, seed=21)
    t = 0.9
    rng = np.random.default_rng(22)
    b = rng.standard_normal(30) * 10.0 ** rng.integers(-6, 6, 30)
    x = rng.standard_normal(30)
    Z = oracle.zmatrix(X, t)
    r = oracle.residual(X, t, x, b=b)
    for j in range(30):
        terms = [Fraction(Z[j, k]) * Fraction(x[k]) for k in range(30)]
        ex = float(Fraction(b[j]) - sum(terms))
        bound = 2.0 ** -52 * abs(ex) + 1e-28 * (abs(b[j]) + float(sum(abs(q) for q in terms)))
        assert abs(r[j] - ex) <= bound, (j, r[j], ex)
    rows = np.array([29, 4, 0])
    assert np.array_equal(oracle.residual(X, t, x, rows, b=b), r[rows])
    # b = 1 reduces to the ones residual exactly
    assert np.array_equal(oracle.residual(X, t, x, b=np.ones(30)), oracle.residual(X, t, x))


@pytest.mark.parametrize("n,m,t", [(200, 3, 0.4), (150, 2, 3.0)])
def test_weighting_solve_general_rhs_vs_lapack(n, m, t):
    # Weighting.solve(b) = Z^{-1} b against LAPACK on numpy's Z, for b far from 1
    X = W.gaussian(n, m, seed=n + m)
    s = oracle.weighting(X, t)
    b = np.random.default_rng(23).standard_normal(n) * 1e3
    x = s.solve(b)
    Z = np.exp(-t * scipy.spatial.distance.cdist(X, X))
    xr = scipy.linalg.solve(Z, b, assume_a="pos")
    ev = np.linalg.eigvalsh(Z)
    # both answers lie within cond * u of Z^{-1} b (scaled by |x|)
    assert np.abs(x - xr).max() <= 50 * (ev[-1] / ev[0]) * 2.0 ** -53 * np.abs(xr).max()
    # the refined answer's Dot2 residual is at unit roundoff of |Z||x| + |b|
    scale = np.abs(Z) @ np.abs(x) + np.abs(b)
    assert np.all(np.abs(oracle.residual(X, t, x, b=b)) <= 4 * 2.0 ** -53 * scale)


def _kgon_parts(k, t):
    q = np.exp(-t)
    S = 1 + sum(np.exp(-2 * t * np.sin(np.pi * j / k)) for j in range(1, k))
    wc = (S - k * q) / (S - k * q * q)
    wr = (1 - q) / (S - k * q * q)
    return q, S, wc, wr


@pytest.mark.parametrize("k,t", [(6, 0.5), (8, 0.7), (12, 1.0), (24, 0.9)])
def test_kappa_M_kgon_closed_form(k, t):
    # below t_+ the centre weight is negative; |w|^T Z |w| over centre and ring is
    # w_c^2 + 2 k |w_c| w_r e^{-t} + k S w_r^2 (each ring row sums to S over the ring)
    q, S, wc, wr = _kgon_parts(k, t)
    assert wc < 0  # t below the k-gon's cutoff
    kappa = (wc * wc + 2 * k * abs(wc) * wr * q + k * S * wr * wr) / abs(wc + k * wr)
    s = oracle.weighting(W.centre_kgon(k), t)
    assert oracle.kappa_M(s) == pytest.approx(kappa, rel=1e-12)
    assert kappa > 1.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kappa_M_is_one_for_nonnegative_weights(seed):
    # w >= 0 gives |w| = w and w^T Z w = 1^T w (the q = 2 diversity identity)
    X = W.gaussian(120, 3, seed=30 + seed)
    s = oracle.weighting(X, oracle.t_bound(X))
    assert s.min_w >= 0
    assert oracle.kappa_M(s) == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("n,m,t", [(250, 3, 0.3), (180, 2, 1.5)])
def test_kappa_M_vs_numpy(n, m, t):
    # with negative weights (t well below t_+) against numpy's own |w|^T Z |w| / |M|
    X = W.gaussian(n, m, seed=40 + n)
    s = oracle.weighting(X, t)
    assert s.min_w < 0
    Z = np.exp(-t * scipy.spatial.distance.cdist(X, X))
    aw = np.abs(s.w)
    ref = float(aw @ Z @ aw) / abs(float(np.sum(s.w)))
    assert oracle.kappa_M(s) == pytest.approx(ref, rel=1e-11)
    assert oracle.kappa_M(s) > 1.0
