"""The metric workload at its full size (n = 32768, m = 3, Gaussian cloud at its
cutoff scale t*), in the launch configuration the benchmark times, checked
against the CPU oracle on sampled outputs it can compute one by one.

* the FP32-factor + refinement solve: oracle residual rows, the device's own
  residual, and agreement with the FP64 dense comparator on the same GPU; the
  same checks at t*/4, t*/2, 2 t* and t_b, and on the anisotropic cloud with
  covariance diag(1, 1/2, 1/4);
* the FP64 matrix-free product Z v: sampled rows against the oracle's row
  products, to the rounding bound of an n-term FP64 sum;
* the FP32 tile generator: every entry among 384 sampled points against the
  oracle's FP64 Z, to a few FP32 ulps.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

N, M_DIM, SEED = 32768, 3, 0
U32 = 2.0 ** -24
U64 = 2.0 ** -53


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.fixture(scope="module")
def workload():
    X = W.gaussian(N, M_DIM, seed=SEED)
    t = float(W.gaussian_cutoff_estimate(N, M_DIM))
    return X, t, dev(X)


def test_metric_solve_sampled_rows(mag, workload):
    X, t, Xd = workload
    res = mag.weighting(Xd, t, solver="fp32_ir")
    w = res.w.cpu().numpy()
    rows = np.random.default_rng(7).choice(N, size=256, replace=False)
    r = np.abs(oracle.residual(X, t, w, rows)).max()
    print(f"n={N} t={t:.6f}: sampled oracle residual {r:.3e}, device {res.info['resid_inf']:.3e}, "
          f"outer={res.info['outer_iters']} gmres={res.info['gmres_iters']} M={res.info['magnitude']:.12g}")
    assert r <= 1e-12
    assert res.info["resid_inf"] <= 1e-12
    assert res.info["argmin_w"] == int(np.argmin(w))
    # the FP64 dense comparator reaches the same weighting
    dense = mag.weighting(Xd, t, solver="fp64_dense")
    wd = dense.w.cpu().numpy()
    assert np.abs(oracle.residual(X, t, wd, rows)).max() <= 1e-12
    assert np.abs(w - wd).max() <= 1e-9 * np.abs(wd).max()
    assert abs(res.info["magnitude"] - dense.info["magnitude"]) <= 1e-10 * abs(dense.info["magnitude"])


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


@pytest.mark.parametrize("scale", [0.25, 0.5, 2.0, "t_b"])
def test_metric_t_sweep_sampled_rows(mag, workload, scale):
    # the metric cloud at t*/4, t*/2, 2 t* and t_b = log(n - 1)/d_min (d_min from the oracle)
    X, tstar, Xd = workload
    t = oracle.t_bound(X) if scale == "t_b" else tstar * scale
    res = _solve_and_check_rows(mag, X, Xd, t, seed=11)
    if scale == "t_b":
        # t_+ <= t_b (the elementary bound of Sections 1 and 2), so w >= 0 there
        assert res.info["min_w"] >= 0


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
