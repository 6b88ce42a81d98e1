"""Solve-level parity: mag_weighting / mag_magnitude (FP32 MFMA factor + FP64
GMRES refinement, and the FP64 dense comparator) against the CPU oracle.

Acceptance (the method's target): ||1 - Z w||_inf <= 1e-12 with Z evaluated in
FP64 by the oracle (Dot2), and |M - M_oracle| / |M_oracle| <= 1e-10 wherever
cond(Z) < 1e10 and 2 u kappa_M <= 1e-11 (beyond that no two correct FP64 codes
need agree to 1e-10).
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


def check_against_oracle(X, t, w, M_gpu=None, resid_tol=1e-12, m_tol=1e-10):
    ref = oracle.weighting(X, t)
    r = oracle.residual(X, t, w)
    assert np.abs(r).max() <= resid_tol, f"residual {np.abs(r).max():.3e}"
    M = float(np.sum(w)) if M_gpu is None else M_gpu
    kM = oracle.kappa_M(ref)
    errM = abs(M - ref.M) / abs(ref.M)
    if 2 * U64 * kM <= 1e-11:
        assert errM <= m_tol, f"M rel err {errM:.3e} (kappa_M {kM:.3e})"
    else:
        assert errM <= 8 * U64 * kM + m_tol
    return ref, errM


SOLVE_CASES = [
    # (name, X builder, t builder)
    ("uniform512_tb", lambda: W.uniform_square(512, seed=0), lambda X: oracle.t_bound(X)),
    ("gauss700_tstar", lambda: W.gaussian(700, 3, seed=1), lambda X: W.gaussian_cutoff_estimate(700, 3)),
    ("gauss1000_tstar_over4", lambda: W.gaussian(1000, 3, seed=2), lambda X: W.gaussian_cutoff_estimate(1000, 3) / 4),
    ("gauss1024_m8_t1", lambda: W.gaussian(1024, 8, seed=3), lambda X: 1.0),
    ("mixture1500_t30", lambda: W.gaussian_mixture(1500, 3, seed=4), lambda X: 30.0),
    ("torus2000_t2", lambda: W.noisy_torus(2000, seed=5), lambda X: 2.0),
    ("z2rect1300_t1", lambda: W.z2_rectangles(1300, seed=6, draws=2000), lambda X: 1.0),
    ("gauss257_m2_t05", lambda: W.gaussian(257, 2, seed=7), lambda X: 0.5),
]


@pytest.mark.parametrize("name,mkX,mkt", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
@pytest.mark.parametrize("solver", ["fp32_ir", "fp64_dense", "fp64_chol"])
def test_weighting_parity(mag, name, mkX, mkt, solver):
    X = mkX()
    t = float(mkt(X))
    res = mag.weighting(dev(X), t, solver=solver)
    w = res.w.cpu().numpy()
    ref, errM = check_against_oracle(X, t, w, M_gpu=res.info["magnitude"])
    # the device's own residual estimate agrees with the oracle's
    if solver == "fp32_ir":
        assert res.info["resid_inf"] <= 1e-12
    assert res.info["argmin_w"] == int(np.argmin(w))
    assert res.info["min_w"] == w.min()
    tol_w, _ = w_tolerance(X, t, w, ref)
    dw = np.abs(w - ref.w).max()
    print(f"{name} {solver}: t={t:.4g} relerr_w={dw / np.abs(ref.w).max():.2e} "
          f"(tol {tol_w / np.abs(ref.w).max():.1e}) relerr_M={errM:.2e} "
          f"outer={res.info['outer_iters']} gmres={res.info['gmres_iters']}")
    assert dw <= tol_w


def test_magnitude_entry_point(mag):
    X = W.gaussian(600, 3, seed=9)
    t = 2.0
    M = mag.magnitude(dev(X), t)
    assert abs(M - oracle.magnitude(X, t)) / abs(M) <= 1e-10


def test_single_point(mag):
    res = mag.weighting(dev(np.array([[0.5, 0.25]])), 3.0)
    assert res.w.cpu().numpy().tolist() == [1.0]
    assert res.info["magnitude"] == 1.0


@pytest.mark.parametrize("t", [0.1, 1.0, 10.0])
def test_two_points_closed_form(mag, t):
    X = np.array([[0.0, 0.0, 0.0], [0.3, 0.4, 1.2]])
    d = 1.3
    w = mag.weighting(dev(X), t).w.cpu().numpy()
    assert np.allclose(w, 1.0 / (1.0 + np.exp(-t * d)), rtol=1e-13)


def test_collinear_closed_form(mag):
    X = W.collinear(900, 3, seed=2)
    t = 0.7
    w = mag.weighting(dev(X), t).w.cpu().numpy()
    s = np.linalg.norm(X - X[0], axis=1)
    order = np.argsort(s)
    g = np.diff(s[order])
    assert abs(w.sum() - (1 + np.tanh(t * g / 2).sum())) <= 1e-9


def test_duplicates_rejected(mag):
    X = W.gaussian(300, 3, seed=1)
    X[17] = X[200]
    with pytest.raises(mag.MagError) as e:
        mag.weighting(dev(X), 1.0)
    assert e.value.code == -2


@pytest.mark.parametrize("solver", ["fp32_ir", "fp64_dense", "fp64_chol", "auto"])
@pytest.mark.parametrize("pair", [(3, 4), (5, 1000), (1299, 0)])
def test_duplicates_rejected_every_solver(mag, solver, pair):
    # the FP32 path finds coincident points inside its tile generator: same tile,
    # tiles far apart, and the last row against the first
    X = W.gaussian(1300, 2, seed=4)
    X[pair[0]] = X[pair[1]]
    with pytest.raises(mag.MagError) as e:
        mag.weighting(dev(X), 2.0, solver=solver)
    assert e.value.code == -2


@pytest.mark.parametrize("t", [0.0, -1.0, float("nan"), float("inf")])
def test_bad_scale_rejected(mag, t):
    with pytest.raises(mag.MagError) as e:
        mag.weighting(dev(W.gaussian(10, 2)), t)
    assert e.value.code == -1


def test_nonfinite_points_rejected(mag):
    X = W.gaussian(50, 2)
    X[3, 1] = np.nan
    with pytest.raises(mag.MagError) as e:
        mag.weighting(dev(X), 1.0)
    assert e.value.code == -1


def test_noconv_reported(mag):
    X = W.gaussian(500, 3, seed=3)
    res = mag.weighting(dev(X), 1.0, max_outer=1, max_gmres=1, raise_on_noconv=False)
    assert res.info["status"] == -3


@pytest.mark.parametrize("solver", ["fp32_ir", "fp64_chol"])
def test_repeat_is_deterministic(mag, solver):
    # fixed-order reductions and no atomics in any sum: bit-identical reruns
    X = W.gaussian(900, 3, seed=4)
    a = mag.weighting(dev(X), 3.0, solver=solver).w.cpu().numpy()
    b = mag.weighting(dev(X), 3.0, solver=solver).w.cpu().numpy()
    assert np.array_equal(a, b)


def test_ill_conditioned_small_t(mag):
    # t -> 0 makes Z nearly 11^T (cond ~ 6e8 here); LAPACK's FP32 Cholesky breaks
    # down on it.  Whether or not the FP32 factor needs the diagonal shift, GMRES
    # with FP64 residuals must still reach the unshifted weighting.
    X = W.gaussian(400, 3, seed=8)
    t = 1e-5
    res = mag.weighting(dev(X), t, max_outer=20, max_gmres=400)
    w = res.w.cpu().numpy()
    print("small-t case:", {k: res.info[k] for k in ("shifted", "shift", "outer_iters", "gmres_iters")})
    check_against_oracle(X, t, w, M_gpu=res.info["magnitude"])


def test_autotune_panel_width_and_table_file(mag, tmp_path):
    # both panel widths give a valid preconditioner; the autotuner keeps the faster
    X = W.gaussian(3000, 3, seed=31)
    t = W.gaussian_cutoff_estimate(3000, 3)
    for nb in (256, 512):
        mag.tune_panel(len(X), nb)
        res = mag.weighting(dev(X), t)
        check_against_oracle(X, t, res.w.cpu().numpy(), M_gpu=res.info["magnitude"])
    nb, ms = mag.autotune(dev(X), t, reps=2)
    assert nb in (256, 512) and all(v > 0 for v in ms)
    assert nb == (256 if ms[0] < ms[1] else 512)
    path = str(tmp_path / "tune.json")
    mag.tune_save(path)
    mag.tune_panel(len(X), 0)
    mag.tune_load(path)
    text = open(path).read()
    assert '"panel"' in text and str(nb) in text
    res = mag.weighting(dev(X), t)
    check_against_oracle(X, t, res.w.cpu().numpy(), M_gpu=res.info["magnitude"])
    print(f"autotune n=3000: picked {nb}, ms(256, 512) = {ms}")
    with pytest.raises(mag.MagError):
        mag.tune_panel(len(X), 384)


@pytest.mark.parametrize("n,m,t", [(3000, 3, 2.0), (2048, 8, 1.0), (1500, 2, 20.0)])
def test_fp32_ir_inner_fp32_products(mag, n, m, t):
    # FP32 entries inside GMRES only; the FP64 residual decides convergence
    X = W.gaussian(n, m, seed=31)
    res = mag.weighting(dev(X), t, solver="fp32_ir", inner_prec="fp32", max_outer=20)
    w = res.w.cpu().numpy()
    assert np.abs(oracle.residual(X, t, w)).max() <= 1e-12
    ref = mag.weighting(dev(X), t, solver="fp32_ir").w.cpu().numpy()
    assert np.abs(w - ref).max() <= 1e-10 * np.abs(ref).max()


def test_inner_prec_rejected_value(mag):
    with pytest.raises(ValueError):
        mag.weighting(dev(W.gaussian(10, 2)), 1.0, inner_prec="fp16")
