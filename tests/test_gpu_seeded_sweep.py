"""A seeded sweep over sizes, dimensions, scales and solvers, each case against
the CPU oracle: sizes on and around every tile edge of the kernels (1, 2, 3, 127,
128, 129, 255, 256, 257, 511, 513, 767, 1025, 1279), dimensions from 1 to 30
(the generic paths above 16), scales from a tenth of to ten times the cloud's
Gaussian cutoff estimate.  Acceptance as in the other parity tests: the oracle's
Dot2 residual on every row <= 1e-12, M to 1e-10 where kappa_M allows it, and w
elementwise within the residual-derived bound."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from parity_util import w_tolerance

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
SIZES = [1, 2, 3, 127, 128, 129, 255, 256, 257, 511, 513, 767, 1025, 1279]
DIMS = [1, 2, 3, 4, 7, 8, 16, 17, 30]


def _cases():
    rng = np.random.default_rng(20261203)
    out = []
    for i in range(36):
        n = int(SIZES[i % len(SIZES)])
        m = int(DIMS[rng.integers(len(DIMS))])
        solvers = ["fp32_ir", "fp64_dense", "auto"]
        if m <= 16 and n >= 4:
            solvers += ["hodlr"]
        if m <= 16 and n >= 200:
            solvers += ["hss"]
        solver = solvers[rng.integers(len(solvers))]
        scale = float(10.0 ** rng.uniform(-1.0, 1.0))
        kind = ["gauss", "mixture", "uniform"][rng.integers(3)]
        out.append((i, n, m, solver, scale, kind))
    return out


CASES = _cases()


def _points(n, m, kind, seed):
    if kind == "mixture" and n >= 5:
        return W.gaussian_mixture(n, m, seed=seed)
    if kind == "uniform":
        return np.random.default_rng(seed).random((n, m))
    return W.gaussian(n, m, seed=seed)


@pytest.mark.parametrize("i,n,m,solver,scale,kind", CASES,
                         ids=[f"{c[0]}-n{c[1]}-m{c[2]}-{c[3]}-{c[5]}" for c in CASES])
def test_seeded_case_against_oracle(mag, i, n, m, solver, scale, kind):
    X = _points(n, m, kind, seed=100 + i)
    t = scale * float(W.gaussian_cutoff_estimate(max(n, 2), m))
    kw = {}
    if solver in ("hodlr", "hss"):
        kw = dict(max_outer=30, max_gmres=600, gmres_restart=100)
    res = mag.weighting(torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0"), t, solver=solver, **kw)
    w = res.w.cpu().numpy()
    ref = oracle.weighting(X, t)
    r = float(np.abs(oracle.residual(X, t, w)).max())
    assert r <= 1e-12, (r, n, m, solver, t)
    kM = oracle.kappa_M(ref)
    errM = abs(res.info["magnitude"] - ref.M) / abs(ref.M)
    if 2 * U64 * kM <= 1e-11:
        assert errM <= 1e-10, (errM, kM)
    else:
        assert errM <= 8 * U64 * kM + 1e-10
    if n >= 2:
        tol, _ = w_tolerance(X, t, w, ref)
        assert np.abs(w - ref.w).max() <= tol
    assert res.info["argmin_w"] == int(np.argmin(w))
