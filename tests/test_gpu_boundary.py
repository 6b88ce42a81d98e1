"""Boundary behaviour of the C ABI on the GPU: the diagnostics of mag_info
(backward error, condition estimate), the workspace cap (MAG_ENOMEM), the
solver MAG_AUTO picks, and point dimensions above 16 (the paper's experiments
use m in {3, 10, 30, 100}, Section 4.3)."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("solver", ["fp32_ir", "fp64_dense", "hodlr", "hss"])
def test_backward_error_and_cond_estimate(mag, solver):
    X = W.gaussian(700, 3, seed=3)
    t = W.gaussian_cutoff_estimate(700, 3) / 2
    res = mag.weighting(dev(X), t, solver=solver, diag=mag.DIAG_BACKWARD | mag.DIAG_COND)
    info = res.info
    w = res.w.cpu().numpy()
    Z = oracle.zmatrix(X, t)
    eta = info["resid_inf"] / (np.abs(Z).sum(axis=1).max() * np.abs(w).max() + 1.0)
    assert info["backward_err"] == pytest.approx(eta, rel=1e-12)
    ev = np.linalg.eigvalsh(Z)
    cond = ev[-1] / ev[0]
    print(f"{solver}: backward_err {info['backward_err']:.3e} cond_est {info['cond_est']:.6g} (eigvalsh {cond:.6g})")
    # Lanczos Ritz values lie inside the spectrum: the estimate approaches cond from below
    assert cond * (1 - 1e-2) <= info["cond_est"] <= cond * (1 + 1e-5)
    assert info["solver"] == mag.SOLVERS[solver]


def test_diagnostics_off_by_default(mag):
    X = W.gaussian(300, 3, seed=4)
    info = mag.weighting(dev(X), 2.0).info
    assert info["backward_err"] == 0.0 and info["cond_est"] == 0.0


def test_workspace_cap_gives_enomem(mag):
    ctx = mag.Context(0)
    X = dev(W.gaussian(2000, 3, seed=5))
    ctx.set_workspace_limit(1 << 20)
    with pytest.raises(mag.MagError) as e:
        mag.weighting(X, 2.0, ctx=ctx)
    assert e.value.code == -4
    assert ctx.workspace_bytes() <= 1 << 20
    with pytest.raises(mag.MagError) as e:
        mag.weighting(X, 2.0, ctx=ctx, solver="hodlr")
    assert e.value.code == -4
    ctx.set_workspace_limit(0)
    res = mag.weighting(X, 2.0, ctx=ctx)
    assert res.info["resid_inf"] <= 1e-12
    held = ctx.workspace_bytes()
    # a cap at what is held lets a same-size solve run again without growing anything
    ctx.set_workspace_limit(held)
    assert mag.weighting(X, 2.0, ctx=ctx).info["resid_inf"] <= 1e-12
    ctx.close()


def test_workspace_cap_from_environment():
    code = ("import sys, torch; sys.path.insert(0, %r); import numpy as np, workloads as W;"
            "import paper_2607_23354_amd as mag\n"
            "X = torch.from_numpy(W.gaussian(2000, 3, seed=5)).to('cuda:0')\n"
            "try:\n    mag.weighting(X, 2.0)\nexcept mag.MagError as e:\n    print('code', e.code)\n"
            "else:\n    print('code', 0)\n") % ROOT
    env = dict(os.environ, MAG_WORKSPACE_LIMIT="1M")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=110)
    assert "code -4" in out.stdout, out.stdout + out.stderr


def test_auto_picks_dense_factor_below_crossover(mag):
    X = W.gaussian(3000, 3, seed=6)
    res = mag.weighting(dev(X), 3.0)
    assert res.info["solver"] == mag.SOLVERS["fp32_ir"]
    assert np.abs(oracle.residual(X, 3.0, res.w.cpu().numpy())).max() <= 1e-12


def test_auto_picks_hodlr_above_crossover(mag):
    # the large torus workload at n = 131072: AUTO takes the HODLR preconditioner
    n, t = 131072, 2.0
    X = W.noisy_torus(n, seed=0)
    res = mag.weighting(dev(X), t)
    info = res.info
    rows = np.random.default_rng(6).choice(n, size=128, replace=False)
    r = np.abs(oracle.residual(X, t, res.w.cpu().numpy(), rows)).max()
    print(f"auto n={n}: solver {mag.SOLVER_NAMES[info['solver']]} resid {info['resid_inf']:.3e} sampled {r:.3e} "
          f"gmres {info['gmres_iters']}")
    assert info["solver"] == mag.SOLVERS["hodlr"]
    assert info["resid_inf"] <= 1e-12 and r <= 1e-12


@pytest.mark.parametrize("m", [30, 100])
def test_fp32_ir_high_dimension(mag, m):
    # the paper's high-dimensional Gaussian experiments, at the cutoff law's scale
    n = 2000
    X = W.gaussian(n, m, seed=m)
    t = float(W.gaussian_cutoff_estimate(n, m))
    res = mag.weighting(dev(X), t, solver="fp32_ir")
    w = res.w.cpu().numpy()
    ref = oracle.weighting(X, t)
    r = np.abs(oracle.residual(X, t, w)).max()
    errM = abs(res.info["magnitude"] - ref.M) / abs(ref.M)
    relw = np.abs(w - ref.w).max() / np.abs(ref.w).max()
    print(f"m={m}: t={t:.4f} resid {r:.3e} relerr_M {errM:.3e} relerr_w {relw:.3e}")
    assert r <= 1e-12 and errM <= 1e-10 and relw <= 1e-10


@pytest.mark.parametrize("m", [30, 100])
def test_adjoint_high_dimension(mag, m):
    # (D o Z) v and the gradient in X beyond 16 dimensions, against the oracle
    n = 600
    X = W.gaussian(n, m, seed=m + 1)
    t = float(W.gaussian_cutoff_estimate(n, m))
    v = np.random.default_rng(m).standard_normal(n)
    y = mag.dzmatvec(dev(X), t, dev(v)).cpu().numpy()
    y_ref = oracle.dzmatvec(X, t, v)
    scale = oracle.dzmatvec(X, t, np.abs(v))
    assert np.all(np.abs(y - y_ref) <= 64 * 2.0 ** -53 * scale)
    gw = np.random.default_rng(m + 2).standard_normal(n)
    Xd = dev(X).requires_grad_(True)
    td = torch.tensor(t, dtype=torch.float64, device="cuda:0", requires_grad=True)
    w, M = mag.MagnitudeFn.apply(Xd, td)
    (M + (w * dev(gw)).sum()).backward()
    dt_ref, dX_ref, sol = oracle.grad(X, t, gM=1.0, gw=gw)
    assert abs(td.grad.item() - dt_ref) <= 1e-10 * abs(dt_ref)
    err = np.abs(Xd.grad.cpu().numpy() - dX_ref).max() / np.abs(dX_ref).max()
    print(f"m={m}: dt err {abs(td.grad.item() - dt_ref) / abs(dt_ref):.2e} dX err {err:.2e}")
    assert err <= 1e-10


def test_spin_limit_forces_the_substitution_timeout(mag):
    # The sync-free triangular solves give up after a bounded number of polls and
    # report MAG_EINTERNAL.  A limit of one poll forces that path from the host:
    # every kernel still finishes (a timed-out workgroup carries on with what it
    # read), the calls fail cleanly, and the context works again at the default.
    n, t = 3000, 2.0
    X = W.gaussian(n, 3, seed=5)
    Xd = dev(X)
    ctx = mag.Context()
    try:
        L, dinv, bd = mag.factor32(Xd, t, ctx=ctx)
        assert bd == 0
        r = dev(np.random.default_rng(3).standard_normal(n))
        z_ref = mag.prec_apply(L, dinv, n, r, ctx=ctx).cpu().numpy()
        ctx.set_spin_limit(1)
        for call in (lambda: mag.prec_apply(L, dinv, n, r, ctx=ctx),
                     lambda: mag.weighting(Xd, t, ctx=ctx),
                     lambda: mag.weighting(Xd, t, ctx=ctx, solver="fp64_chol")):
            with pytest.raises(mag.MagError) as e:
                call()
            assert e.value.code == -6  # MAG_EINTERNAL
        ctx.set_spin_limit(0)
        assert np.array_equal(mag.prec_apply(L, dinv, n, r, ctx=ctx).cpu().numpy(), z_ref)
        w = mag.weighting(Xd, t, ctx=ctx).w.cpu().numpy()
        assert np.abs(oracle.residual(X, t, w)).max() <= 1e-12
        with pytest.raises(mag.MagError):
            ctx.set_spin_limit(-1)
    finally:
        ctx.close()
