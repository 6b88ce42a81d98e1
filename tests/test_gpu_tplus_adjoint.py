"""GPU parity of the cutoff search (mag_tplus) and of the adjoint
(mag_dwdt, mag_weighting_fwd/vjp, MagnitudeFn) against the CPU oracle,
closed forms and finite differences."""
import numpy as np
import pytest
import scipy.optimize
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def kgon_root(k):
    def f(t):
        S = 1 + sum(np.exp(-2 * t * np.sin(np.pi * j / k)) for j in range(1, k))
        return S - k * np.exp(-t)
    return scipy.optimize.brentq(f, 0.05, 10.0, xtol=1e-15, rtol=1e-15)


# ------------------------------------------------------------------ t_+

@pytest.mark.parametrize("k", [6, 8, 12, 24])
@pytest.mark.parametrize("newton,method", [(True, "bisection"), (False, "bisection"), (False, "ridders")])
def test_tplus_kgon_closed_form(mag, k, newton, method):
    root = kgon_root(k)
    r = mag.tplus(dev(W.centre_kgon(k)), rtol=1e-7, newton=newton, method=method)
    assert r.info["no_sign_change"] == 0
    assert root <= r.t_plus * (1 + 1e-12)
    assert (r.t_plus - root) / root <= 2e-7, (r.t_plus, root, r.info)
    assert r.info["min_w"] >= 0
    assert r.w is not None and r.w.cpu().numpy().min() >= 0


def test_tplus_collinear_and_tiny(mag):
    # points on a line: w > 0 at every t (Z^{-1} is tridiagonal, weights are
    # sums of tanh terms).  The scan stays on [t_b 1e-3, t_b]: far below it the
    # interior weights (~ t * gap) fall under the FP64 error bound of any solve,
    # so their sign is not determined by the arithmetic.
    rng = np.random.default_rng(4)
    s_pos = np.linspace(0.0, 1.0, 300) + rng.random(300) * (0.1 / 300)
    direction = np.array([0.48, -0.6, 0.64])
    X = np.ascontiguousarray(s_pos[:, None] * direction[None, :] + np.array([1.0, 2.0, -0.5]))
    r = mag.tplus(dev(X), max_extend=0)
    assert r.info["no_sign_change"] == 1 and r.t_plus == 0.0
    assert oracle.tplus(X, max_extend=0).no_sign_change
    for X in (np.zeros((1, 2)), np.array([[0.0, 0.0], [1.0, 2.0]])):
        r = mag.tplus(dev(X))
        assert r.info["no_sign_change"] == 1 and r.t_plus == 0.0


@pytest.mark.parametrize("method", ["bisection", "ridders"])
@pytest.mark.parametrize("n,seed", [(300, 0), (777, 1), (1100, 2)])
def test_tplus_vs_oracle_mixture(mag, n, seed, method):
    X = W.gaussian_mixture(n, 3, seed=seed)
    r = mag.tplus(dev(X), method=method)
    ref = oracle.tplus(X)
    assert r.info["no_sign_change"] == 0 and not ref.no_sign_change
    # both are upper ends of brackets of relative width <= 1e-6 around the same root
    assert abs(r.t_plus - ref.t_plus) / ref.t_plus <= 2.5e-6, (r.info, ref.t_plus)
    assert r.info["d_min"] == oracle.dmin(X)
    # brute-force signs (oracle solves) around the GPU's cutoff
    assert oracle.weighting(X, r.t_plus * (1 + 1e-5)).min_w >= 0
    assert oracle.weighting(X, r.t_plus * (1 - 1e-5)).min_w < 0
    print(f"n={n}: t+={r.t_plus:.8g} oracle={ref.t_plus:.8g} solves gpu={r.info['solves']} "
          f"newton={r.info['newton_steps']} oracle solves={ref.solves}")


def test_tplus_newton_saves_solves(mag):
    X = W.gaussian_mixture(600, 3, seed=7)
    a = mag.tplus(dev(X), newton=True)
    b = mag.tplus(dev(X), newton=False)
    assert abs(a.t_plus - b.t_plus) / b.t_plus <= 2.5e-6
    assert a.info["solves"] < b.info["solves"]


def test_tplus_ridders_vs_bisection(mag):
    # Ridders' interpolation (no derivative) against plain bisection: the same
    # cutoff, in fewer solves on a smooth min w(t)
    for seed in (7, 9):
        X = W.gaussian_mixture(600, 3, seed=seed)
        a = mag.tplus(dev(X), method="ridders")
        b = mag.tplus(dev(X), newton=False)
        print(seed, a.t_plus, a.info["solves"], a.info["newton_steps"], b.t_plus, b.info["solves"])
        assert abs(a.t_plus - b.t_plus) / b.t_plus <= 2.5e-6
        assert a.info["newton_steps"] > 0
        assert a.info["solves"] <= b.info["solves"]
    with pytest.raises(ValueError):
        mag.tplus(dev(X), method="brent")


def test_tplus_scaling(mag):
    X = W.gaussian(400, 3, seed=3)
    lam = 2.5
    a = mag.tplus(dev(X)).t_plus
    b = mag.tplus(dev(lam * X)).t_plus
    assert abs(b * lam - a) / a <= 3e-6


def test_tplus_resume_bracket(mag):
    X = W.gaussian_mixture(500, 3, seed=8)
    full = mag.tplus(dev(X))
    lo, hi = full.info["t_bracket_lo"], full.info["t_bracket_hi"]
    r = mag.tplus(dev(X), t_lo=lo * 0.9, t_hi=hi * 1.1)
    assert abs(r.t_plus - full.t_plus) / full.t_plus <= 2.5e-6
    assert r.info["solves"] < full.info["solves"]


# ------------------------------------------------------------------ derivatives

@pytest.mark.parametrize("n,m,t", [(300, 3, 2.0), (700, 8, 1.0), (257, 2, 0.5)])
def test_dzmatvec_vs_oracle(mag, n, m, t):
    X = W.gaussian(n, m, seed=n)
    v = np.random.default_rng(1).standard_normal(n)
    y = mag.dzmatvec(dev(X), t, dev(v)).cpu().numpy()
    y_ref = oracle.dzmatvec(X, t, v)
    scale = oracle.dzmatvec(X, t, np.abs(v))
    assert np.all(np.abs(y - y_ref) <= 64 * 2.0 ** -53 * scale)


@pytest.mark.parametrize("n,m,t", [(400, 3, 3.0), (600, 8, 1.0)])
def test_dwdt_vs_oracle(mag, n, m, t):
    X = W.gaussian(n, m, seed=n + 5)
    w, d = mag.dwdt(dev(X), t)
    w, d = w.cpu().numpy(), d.cpu().numpy()
    sol = oracle.weighting(X, t)
    d_ref = oracle.dw_dt(sol)
    # dw/dt solves Z d = g with g = (D o Z) w.  (a) The device's d satisfies the
    # oracle's equation up to its own solve tolerance (1e-12 relative to g) plus the
    # change of g that its w makes: |g_gpu - g_ref| <= (D o Z)|w - w_ref|.
    g_ref = oracle.dzmatvec(X, t, sol.w)
    r1 = oracle.residual(X, t, d, b=g_ref)
    dg = oracle.dzmatvec(X, t, np.abs(w - sol.w))
    assert np.all(np.abs(r1) <= 1e-12 * max(1.0, np.abs(g_ref).max()) + 2 * dg + 1e-15 * np.abs(g_ref).max())
    # (b) then |d - d_ref|_2 <= (|r1|_2 + |r2|_2) / lambda_min, r2 the oracle's own
    # residual (twice that, for the estimate of lambda_min)
    r2 = oracle.residual(X, t, d_ref, b=g_ref)
    _, lmin, _ = oracle.cond_estimate(sol)
    bound = 2 * (np.linalg.norm(r1) + np.linalg.norm(r2)) / lmin
    err = np.abs(d - d_ref).max()
    print(f"dw/dt n={n}: |d - d_ref|_inf / |d_ref|_inf = {err / np.abs(d_ref).max():.2e} "
          f"(bound {bound / np.abs(d_ref).max():.2e})")
    assert err <= max(bound, 1e-14 * np.abs(d_ref).max())


@pytest.mark.parametrize("with_gw", [False, True])
def test_vjp_vs_oracle(mag, with_gw):
    n, m, t = 1024, 8, 1.0  # the adjoint workload's oracle size
    X = W.gaussian(n, m, seed=0)
    gw = np.random.default_rng(1).standard_normal(n) if with_gw else None
    Xd = dev(X).requires_grad_(True)
    td = torch.tensor(t, dtype=torch.float64, device="cuda:0", requires_grad=True)
    w, M = mag.MagnitudeFn.apply(Xd, td)
    loss = M if gw is None else M + (w * dev(gw)).sum()
    loss.backward()
    dt_ref, dX_ref, sol = oracle.grad(X, t, gM=1.0, gw=gw)
    assert abs(M.item() - sol.M) / abs(sol.M) <= 1e-10
    err_t = abs(td.grad.item() - dt_ref) / abs(dt_ref)
    err = np.abs(Xd.grad.cpu().numpy() - dX_ref).max() / np.abs(dX_ref).max()
    print(f"vjp n={n} m={m} gw={with_gw}: dL/dt rel err {err_t:.2e}, dL/dX rel err {err:.2e}, "
          f"kappa_M {oracle.kappa_M(sol):.3g}")
    # the oracle's analytic gradient to 1e-10 where kappa_M allows it (two correct
    # FP64 evaluations may differ by about 2 u kappa_M), else to that bound
    tol = 1e-10 if 2.0 ** -52 * oracle.kappa_M(sol) <= 1e-11 else 1e-10 + 8 * 2.0 ** -53 * oracle.kappa_M(sol)
    assert err_t <= tol
    assert err <= tol, err


def test_two_point_gradient_closed_form(mag):
    X = np.array([[0.1, 0.2, 0.0], [0.9, -0.3, 0.4]])
    d = float(np.linalg.norm(X[0] - X[1]))
    t = 1.7
    Xd = dev(X).requires_grad_(True)
    td = torch.tensor(t, dtype=torch.float64, device="cuda:0", requires_grad=True)
    w, M = mag.MagnitudeFn.apply(Xd, td)
    M.backward()
    assert td.grad.item() == pytest.approx(2 * d * np.exp(-t * d) / (1 + np.exp(-t * d)) ** 2, rel=1e-12)
    g0 = (t / 2) / np.cosh(t * d / 2) ** 2 * (X[0] - X[1]) / d
    assert np.allclose(Xd.grad.cpu().numpy(), [g0, -g0], rtol=1e-11)


def test_vjp_finite_differences_full_size(mag):
    # the adjoint workload at full size: n = 16384, m = 8, X ~ N(0, I), t = 1,
    # gw ~ N(0, 1), gM = 1; central differences with h = 1e-6 in t and along a
    # random direction in X (the solves behind the differences are driven to
    # the FP64 floor so that their noise stays below the tolerance)
    n, m, t, h = 16384, 8, 1.0, 1e-6
    X = W.gaussian(n, m, seed=0)
    gw = np.random.default_rng(1).standard_normal(n)
    Xd = dev(X).requires_grad_(True)
    td = torch.tensor(t, dtype=torch.float64, device="cuda:0", requires_grad=True)
    w, M = mag.MagnitudeFn.apply(Xd, td)
    loss = M + (w * dev(gw)).sum()
    loss.backward()
    wv = w.detach().cpu().numpy()
    # w solves Z w = 1 (sampled rows, oracle Dot2 residual)
    rows = np.random.default_rng(2).choice(n, 64, replace=False)
    assert np.abs(oracle.residual(X, t, wv, rows)).max() <= 1e-12

    def L(Xv, tv):
        r = mag.weighting(dev(Xv), tv, tol=1e-15, raise_on_noconv=False)
        return r.info["magnitude"] + float(gw @ r.w.cpu().numpy())

    fd_t = (L(X, t + h) - L(X, t - h)) / (2 * h)
    V = np.random.default_rng(3).standard_normal((n, m))
    fd_x = (L(X + h * V, t) - L(X - h * V, t)) / (2 * h)
    gX = Xd.grad.cpu().numpy()
    print(f"finite differences n={n}: dL/dt rel {abs(td.grad.item() - fd_t) / abs(fd_t):.2e}, "
          f"directional dL/dX rel {abs(float(np.sum(gX * V)) - fd_x) / abs(fd_x):.2e}")
    # h = 1e-6 central differences: truncation ~h^2, rounding ~u |L| / h
    assert td.grad.item() == pytest.approx(fd_t, rel=1e-6)
    assert float(np.sum(gX * V)) == pytest.approx(fd_x, rel=1e-6)
