"""The benchmark workloads at their full sizes, in the launch configuration the
benchmark times, checked against the CPU oracle.

* the metric workload (Gaussian cloud, n = 32768, m = 3, seed 0) at t*, t*/4,
  t*/2, 2 t* and t_b: w elementwise and M against the oracle's weighting
  (``tests/golden/full_size``, written by ``tests/golden/make_full_size.py``
  from the oracle alone), the oracle's Dot2 residual on every row, the
  device's own residual; at t* also both FP64 dense comparators;
* the Z^2 rectangle workload (n = 8192) at its five scales, the same checks,
  for the FP32 + refinement solve and both FP64 dense comparators;
* the anisotropic cloud with covariance diag(1, 1/2, 1/4): sampled oracle rows;
* the FP64 matrix-free product Z v: sampled rows against the oracle's row
  products, to the rounding bound of an n-term FP64 sum;
* the FP32 tile generator: every entry among 384 sampled points against the
  oracle's FP64 Z, to a few FP32 ulps;
* the preconditioner apply of the refinement at n = 32768: backward error of
  L L^T z = r against its FP32 rounding bound.

Tolerance on w.  Both weightings solve Z w = 1 up to their residuals, so
w_gpu - w_gold = Z^{-1} (r_gold - r_gpu) and
||w_gpu - w_gold||_inf <= ||r_gold - r_gpu||_2 / lambda_min(Z).  The test
takes the larger of 1e-10 ||w||_inf and twice that bound, with ||r_gpu||_2
from the oracle's residual on every row, ||r_gold||_2 <= sqrt(n) times the
stored residual, and lambda_min the oracle's inverse-iteration estimate.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

N, M_DIM, SEED = 32768, 3, 0
U32 = 2.0 ** -24
U64 = 2.0 ** -53
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size")


def golden(key):
    with open(os.path.join(GOLD, "index.json")) as f:
        rec = json.load(f)[key]
    return rec, np.load(os.path.join(GOLD, rec["w_file"]), allow_pickle=False)


def check_vs_golden(X, rec, wg, res, label):
    """The solve's w and M against the oracle's expected values (see the module
    docstring for the tolerance on w); the oracle's Dot2 residual on every row."""
    n = len(X)
    t = rec["t"]
    w = res.w.cpu().numpy()
    r = oracle.residual(X, t, w)
    rinf = float(np.abs(r).max())
    dw = float(np.abs(w - wg).max())
    bound_w = 2.0 * (float(np.linalg.norm(r)) + np.sqrt(n) * rec["resid_inf"]) / rec["lambda_min_est"]
    tol_w = max(1e-10 * float(np.abs(wg).max()), bound_w)
    M = res.info["magnitude"]
    errM = abs(M - rec["M"]) / abs(rec["M"])
    kM = rec["kappa_M"]
    print(f"{label}: t={t:.6g} oracle resid (all rows) {rinf:.3e} device {res.info['resid_inf']:.3e} "
          f"relerr_w={dw / np.abs(wg).max():.3e} (tol {tol_w / np.abs(wg).max():.1e}) relerr_M={errM:.3e} "
          f"kappa_M={kM:.4g} cond~{rec['cond_est']:.3g} outer={res.info['outer_iters']} "
          f"gmres={res.info['gmres_iters']}")
    assert rinf <= 1e-12
    assert res.info["resid_inf"] <= 1e-12
    assert dw <= tol_w
    if rec["cond_est"] < 1e10 and 2 * U64 * kM <= 1e-11:
        assert errM <= 1e-10
    else:
        assert errM <= 8 * U64 * kM + 1e-10
    # the reported minimum is the minimum of the returned w, and the oracle's
    # minimum agrees with it to the tolerance on w
    assert res.info["min_w"] == w.min()
    assert w[res.info["argmin_w"]] == w.min()
    assert abs(w.min() - rec["min_w"]) <= tol_w
    return w, errM, dw / np.abs(wg).max()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.fixture(scope="module")
def workload():
    X = W.gaussian(N, M_DIM, seed=SEED)
    t = float(W.gaussian_cutoff_estimate(N, M_DIM))
    return X, t, dev(X)


METRIC_SCALES = ["tstar", "tstar_over4", "tstar_over2", "tstar_x2", "t_b"]


@pytest.mark.parametrize("scale", METRIC_SCALES)
def test_metric_vs_oracle(mag, workload, scale):
    X, tstar, Xd = workload
    rec, wg = golden(f"gauss_n32768_m3_seed0_{scale}")
    assert rec["n"] == N and rec["m"] == M_DIM
    if scale == "tstar":
        assert rec["t"] == tstar
    res = mag.weighting(Xd, rec["t"], solver="fp32_ir")
    w, _, _ = check_vs_golden(X, rec, wg, res, f"metric n={N} {scale}")
    if scale == "t_b":
        # t_+ <= t_b (the elementary bound of Sections 1 and 2), so w >= 0 there
        assert res.info["min_w"] >= 0
    if scale == "tstar":
        # the FP64 dense comparators (rocSOLVER's and this library's FP64 MFMA
        # factor) reach the same weighting
        for solver in ("fp64_dense", "fp64_chol"):
            dense = mag.weighting(Xd, rec["t"], solver=solver)
            check_vs_golden(X, rec, wg, dense, f"metric n={N} {scale} {solver}")


Z2_SCALES = ["0.25", "0.5", "1", "2", "4"]


@pytest.fixture(scope="module")
def z2_workload():
    X = W.z2_rectangles(8192, seed=0)
    return X, dev(X)


@pytest.mark.parametrize("f", Z2_SCALES)
@pytest.mark.parametrize("solver", ["fp32_ir", "fp64_dense", "fp64_chol"])
def test_z2_rectangles_vs_oracle(mag, z2_workload, f, solver):
    # the lattice workload (n = 8192 unique points of Z^2) at t = f * log(n - 1)/d_min
    X, Xd = z2_workload
    rec, wg = golden(f"z2rect_n8192_seed0_tb_x{f}")
    assert rec["n"] == len(X)
    res = mag.weighting(Xd, rec["t"], solver=solver)
    check_vs_golden(X, rec, wg, res, f"z2 n=8192 t_b x{f} {solver}")


def _solve_and_check_rows(mag, X, Xd, t, seed):
    res = mag.weighting(Xd, t, solver="fp32_ir")
    w = res.w.cpu().numpy()
    rows = np.random.default_rng(seed).choice(len(X), size=128, replace=False)
    r = np.abs(oracle.residual(X, t, w, rows)).max()
    print(f"n={len(X)} t={t:.6f}: sampled oracle residual {r:.3e}, device {res.info['resid_inf']:.3e}, "
          f"outer={res.info['outer_iters']} gmres={res.info['gmres_iters']} shifted={res.info['shifted']} "
          f"M={res.info['magnitude']:.12g}")
    assert r <= 1e-12
    assert res.info["resid_inf"] <= 1e-12
    assert res.info["argmin_w"] == int(np.argmin(w))
    return res


def test_metric_anisotropic_sampled_rows(mag, workload):
    # the same size with covariance diag(1, 1/2, 1/4), at the isotropic cloud's t*
    _, tstar, _ = workload
    X = W.gaussian(N, M_DIM, seed=SEED, diag=(1.0, 0.5, 0.25))
    _solve_and_check_rows(mag, X, dev(X), tstar, seed=12)


def test_metric_zmatvec_sampled_rows(mag, workload):
    X, t, Xd = workload
    v = np.random.default_rng(8).standard_normal(N)
    y = mag.zmatvec(Xd, t, dev(v)).cpu().numpy()
    rows = np.random.default_rng(9).choice(N, size=256, replace=False)
    # the oracle's residual 1 - (Z v)_j gives the row products exactly rounded
    # (Dot2); |Z||v| bounds the rounding of an n-term FP64 sum
    ref = 1.0 - oracle.residual(X, t, v, rows)
    mag_rows = 1.0 - oracle.residual(X, t, np.abs(v), rows)
    err = np.abs(y[rows] - ref)
    assert np.all(err <= 4 * N * U64 * mag_rows + 1e-300)


def test_metric_tile32_sampled_block(mag, workload):
    X, t, Xd = workload
    A = mag.tile32(Xd, t)  # A[j, i] = Z_ij on the lower triangle (i >= j), FP32
    sub = np.sort(np.random.default_rng(10).choice(N, size=384, replace=False))
    idx = torch.from_numpy(sub).to(A.device)
    got = A.index_select(0, idx).index_select(1, idx).cpu().numpy().T.astype(np.float64)  # got[a, b] = Z_{sub a, sub b}
    del A
    torch.cuda.empty_cache()
    Z = oracle.zmatrix(X[sub], t)
    D = oracle.distance_matrix(X[sub])
    lower = np.tril(np.ones_like(Z, dtype=bool))
    # FP32 evaluation of exp(-x), x = t d: x = fl(fl(t) * sqrtf(fl(d^2))) carries up to
    # 3.5 unit roundoffs (t, d^2 halved by the root, the root, the product), so
    # |dZ| <= 3.5 U32 x Z, plus expf's own few units; at this t the far pairs'
    # entries (down to e^-95) fall below FP32's normal range, where the device may
    # flush them to zero: allow that absolute level
    tol = (4 + 4 * t * D) * U32 * Z + 2.0 ** -126
    err = np.abs(got - Z)
    bad = lower & (err > tol)
    assert not bad.any(), (f"{bad.sum()} entries off; worst: Z={Z[bad][:4]} got={got[bad][:4]} "
                           f"t*d={t * D[bad][:4]}")
    assert np.all(np.diag(got) == 1.0)


def test_metric_prec_apply_backward_error(mag, workload):
    # the refinement's preconditioner apply z = (L L^T)^{-1} r at the metric size, in
    # the launch configuration the solve uses (one workgroup per 128-row block, near
    # tiles D_b L(b, b -/+ 1) formed from the factor): L L^T z reproduces r to the
    # rounding of FP32 block inverses and near tiles.  Per block the substitution
    # applies D_b = L_bb^{-1} + E with |E| <~ kappa_b u32 |L_bb^{-1}| (kappa_b the
    # block's condition number) and near tiles rounded to FP32, so every row of
    # L L^T z - r is bounded by a small multiple of 128 kappa_b u32 (|L| |L^T| |z|)
    X, t, Xd = workload
    L, dinv, bd = mag.factor32(Xd, t)
    assert bd == 0
    r = np.random.default_rng(11).standard_normal(N)
    z = mag.prec_apply(L, dinv, N, dev(r))
    U = torch.triu(L[:N, :N]).double()  # the upper triangle holds L^T
    del L
    torch.cuda.empty_cache()
    # kappa_b = max_b ||L_bb||_inf ||D_b||_inf over the 256 diagonal blocks
    kb = 0.0
    for b in range(N // 128):
        Lbb = U[128 * b:128 * (b + 1), 128 * b:128 * (b + 1)].T
        Db = dinv[b].double().T  # dinv[b] holds D_b column-major
        kb = max(kb, float(Lbb.abs().sum(1).max() * Db.abs().sum(1).max()))
    rr = U.T @ (U @ z.unsqueeze(1))
    scale = U.abs().T @ (U.abs() @ z.abs().unsqueeze(1))
    err = (rr.squeeze(1) - dev(r)).abs()
    tol = 16 * 128 * kb * U32 * scale.squeeze(1)
    worst = float((err / scale.squeeze(1)).max())
    print(f"prec apply n={N}: kappa_b={kb:.3g} max |L L^T z - r| / (|L||L^T||z|) = {worst:.3e} "
          f"(bound {16 * 128 * kb * U32:.3e})")
    assert bool((err <= tol).all())
