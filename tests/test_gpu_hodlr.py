"""HODLR-preconditioned solves (MAG_HODLR) against the CPU oracle.

The HODLR factors themselves (tree, bases, ranks) are not unique, so only
the final weighting is compared: ||1 - Z w||_inf <= 1e-12 with Z evaluated by
the oracle in FP64 (Dot2), and the magnitude to 1e-10 where kappa_M allows it
(same acceptance as the dense-factor path).  At the full size (n = 131072,
noisy torus) the oracle checks sampled rows of the residual one by one.
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


CASES = [
    ("torus2000_t05", lambda: W.noisy_torus(2000, seed=5), 0.5, {}),
    ("torus2000_t2", lambda: W.noisy_torus(2000, seed=5), 2.0, {}),
    ("torus2000_t8", lambda: W.noisy_torus(2000, seed=5), 8.0, {}),
    ("gauss3001_tstar", lambda: W.gaussian(3001, 3, seed=11), W.gaussian_cutoff_estimate(3001, 3), {}),
    ("gauss1200_m8_t1", lambda: W.gaussian(1200, 8, seed=12), 1.0, {}),
    ("gauss1500_m2_t05", lambda: W.gaussian(1500, 2, seed=13), 0.5, {}),
    ("mixture2500_t30", lambda: W.gaussian_mixture(2500, 3, seed=14), 30.0, {}),
    ("single_leaf100", lambda: W.gaussian(100, 3, seed=15), 2.0, {}),
    ("two_leaves129", lambda: W.gaussian(129, 3, seed=16), 2.0, {}),
    ("torus2000_leaf32", lambda: W.noisy_torus(2000, seed=5), 2.0, {"leaf": 32}),
    ("torus2000_rank8", lambda: W.noisy_torus(2000, seed=5), 2.0,
     {"max_rank": 8, "oversample": 0, "gmres_restart": 120, "max_gmres": 600, "max_outer": 20}),
    ("torus2000_rank512", lambda: W.noisy_torus(2000, seed=5), 0.5, {"max_rank": 512}),
    ("gauss5000_rank512_tstar", lambda: W.gaussian(5000, 3, seed=17), W.gaussian_cutoff_estimate(5000, 3),
     {"max_rank": 512}),
    # leaves of 129..256 points: batched Cholesky factor and inverse in HBM
    ("single_leaf200_leaf256", lambda: W.gaussian(200, 3, seed=18), 2.0, {"leaf": 256}),
    ("torus3000_leaf256_t05", lambda: W.noisy_torus(3000, seed=5), 0.5, {"leaf": 256}),
    ("torus3000_leaf256_rank64_t2", lambda: W.noisy_torus(3000, seed=5), 2.0,
     {"leaf": 256, "max_rank": 64, "oversample": 0, "gmres_restart": 100, "max_gmres": 400, "max_outer": 30}),
    ("gauss3001_leaf256_tstar", lambda: W.gaussian(3001, 3, seed=11), W.gaussian_cutoff_estimate(3001, 3),
     {"leaf": 256}),
    ("gauss1200_m8_leaf256_t1", lambda: W.gaussian(1200, 8, seed=12), 1.0, {"leaf": 256}),
    ("mixture2500_leaf160_t30", lambda: W.gaussian_mixture(2500, 3, seed=14), 30.0, {"leaf": 160}),
    # range finder with subspace iterations
    ("torus3000_power1_t05", lambda: W.noisy_torus(3000, seed=5), 0.5, {"power_iters": 1}),
    ("torus3000_power1_rank64_t2", lambda: W.noisy_torus(3000, seed=5), 2.0,
     {"power_iters": 1, "max_rank": 64, "oversample": 0, "gmres_restart": 100, "max_gmres": 400}),
    ("gauss3001_power2_leaf256_tstar", lambda: W.gaussian(3001, 3, seed=11), W.gaussian_cutoff_estimate(3001, 3),
     {"power_iters": 2, "leaf": 256}),
    ("gauss1200_m8_power1_t1", lambda: W.gaussian(1200, 8, seed=12), 1.0, {"power_iters": 1}),
    # edges of the new paths: two leaves of 128 and 129 points (the 256 stride for a
    # 129-point leaf), the largest dimension with 256-point leaves, the most
    # subspace iterations, a 5-slab basis (320 columns: a 4-slab and a 1-slab launch)
    ("two_leaves257_leaf256", lambda: W.gaussian(257, 3, seed=19), 2.0, {"leaf": 256}),
    ("gauss2000_m16_leaf256_t1", lambda: W.gaussian(2000, 16, seed=20), 1.0, {"leaf": 256}),
    ("torus2500_power4", lambda: W.noisy_torus(2500, seed=21), 2.0, {"power_iters": 4}),
    ("torus4000_rank256_p16_power1", lambda: W.noisy_torus(4000, seed=22), 2.0,
     {"max_rank": 256, "oversample": 16, "power_iters": 1}),
]


@pytest.mark.parametrize("name,mkX,t,kw", CASES, ids=[c[0] for c in CASES])
def test_hodlr_parity(mag, name, mkX, t, kw):
    X = mkX()
    res = mag.weighting(dev(X), float(t), solver="hodlr", **kw)
    w, ref, errM = check(X, float(t), res)
    tol_w, _ = w_tolerance(X, float(t), w, ref)
    relw = np.abs(w - ref.w).max() / np.abs(ref.w).max()
    assert np.abs(w - ref.w).max() <= tol_w
    print(f"{name}: n={len(X)} t={t:.4g} relerr_w={relw:.2e} (tol {tol_w / np.abs(ref.w).max():.1e}) "
          f"relerr_M={errM:.2e} "
          f"outer={res.info['outer_iters']} gmres={res.info['gmres_iters']}")


def test_hodlr_deterministic(mag):
    X = W.noisy_torus(1500, seed=3)
    a = mag.weighting(dev(X), 1.0, solver="hodlr").w.cpu().numpy()
    b = mag.weighting(dev(X), 1.0, solver="hodlr").w.cpu().numpy()
    assert np.array_equal(a, b)


def test_hodlr_permutation_equivariant(mag):
    # the cluster tree reorders the points; the answer must follow the caller's
    # order.  The two solves use different (equally valid) preconditioners, so
    # they agree to the solve's accuracy, not bitwise.
    X = W.gaussian(900, 3, seed=21)
    p = np.random.default_rng(0).permutation(len(X))
    w = mag.weighting(dev(X), 3.0, solver="hodlr").w.cpu().numpy()
    wp = mag.weighting(dev(X[p]), 3.0, solver="hodlr").w.cpu().numpy()
    assert np.abs(oracle.residual(X[p], 3.0, wp)).max() <= 1e-12
    assert np.abs(wp - w[p]).max() <= 1e-10 * np.abs(w).max()


def test_hodlr_rejects_bad_options(mag):
    X = dev(W.gaussian(300, 3, seed=1))
    with pytest.raises(mag.MagError):
        mag.weighting(X, 1.0, solver="hodlr", leaf=257)
    with pytest.raises(mag.MagError):
        mag.weighting(X, 1.0, solver="hodlr", leaf=1)
    with pytest.raises(mag.MagError):
        mag.weighting(X, 1.0, solver="hodlr", power_iters=5)
    with pytest.raises(mag.MagError):
        mag.weighting(X, 1.0, solver="hodlr", power_iters=-1)
    with pytest.raises(mag.MagError):
        mag.weighting(dev(W.gaussian(300, 17, seed=1)), 1.0, solver="hodlr")


@pytest.mark.parametrize("leaf", [128, 256])
def test_hodlr_duplicates(mag, leaf):
    # two equal points in one leaf: the leaf block is singular (the sweep's or the
    # batched Cholesky's failed pivot)
    X = W.gaussian(400, 3, seed=2)
    X[7] = X[300]
    with pytest.raises(mag.MagError):
        mag.weighting(dev(X), 1.0, solver="hodlr", leaf=leaf)


def test_hodlr_leaf256_matches_leaf128(mag):
    # two different preconditioners of one system: the answers agree to the solves'
    # accuracy, and the one-leaf factor (n <= leaf) is the exact inverse
    X = W.noisy_torus(2500, seed=9)
    a = mag.weighting(dev(X), 2.0, solver="hodlr", leaf=128)
    b = mag.weighting(dev(X), 2.0, solver="hodlr", leaf=256)
    wa, wb = a.w.cpu().numpy(), b.w.cpu().numpy()
    assert np.abs(wa - wb).max() <= 1e-10 * np.abs(wa).max()
    Xs = W.gaussian(250, 3, seed=4)
    one = mag.weighting(dev(Xs), 1.5, solver="hodlr", leaf=256)
    assert one.info["gmres_iters"] <= 2
    assert np.abs(oracle.residual(Xs, 1.5, one.w.cpu().numpy())).max() <= 1e-12


INNER32 = [c for c in CASES if c[0] in ("torus2000_t05", "torus2000_t8", "gauss3001_tstar",
                                        "gauss1200_m8_t1", "torus2000_rank8", "mixture2500_t30")]


@pytest.mark.parametrize("name,mkX,t,kw", INNER32, ids=[c[0] for c in INNER32])
def test_hodlr_inner_fp32_products(mag, name, mkX, t, kw):
    # FP32 entries inside GMRES only: the FP64 residual still decides, so the
    # answer meets the same acceptance as with FP64 inner products
    X = mkX()
    kw = dict(kw)
    kw.setdefault("max_outer", 30)
    kw.setdefault("max_gmres", 600)
    res = mag.weighting(dev(X), float(t), solver="hodlr", inner_prec="fp32", **kw)
    w, ref, errM = check(X, float(t), res)
    print(f"{name} (inner fp32): outer={res.info['outer_iters']} gmres={res.info['gmres_iters']} "
          f"relerr_M={errM:.2e}")
