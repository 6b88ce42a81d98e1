"""Shared tolerance of the GPU parity tests on the weighting w.

Two solutions of Z w = 1 differ by w_a - w_b = Z^{-1} (r_b - r_a), r = 1 - Z w,
so ||w_a - w_b||_inf <= ||r_a - r_b||_2 / lambda_min(Z).  The residuals are the
oracle's Dot2 evaluations on every row; lambda_min comes from the oracle's
inverse iteration (an estimate from above, hence the factor 2)."""
import numpy as np

import oracle


def w_tolerance(X, t, w, ref, floor=1e-10):
    """Largest |w - ref.w| that two solutions with these residuals may show:
    max(floor * ||ref.w||_inf, 2 ||r_w - r_ref||_2 / lambda_min)."""
    r_w = oracle.residual(X, t, w)
    r_ref = oracle.residual(X, t, ref.w)
    _, lmin, _ = oracle.cond_estimate(ref, iters=200, rtol=1e-8)
    bound = 2.0 * float(np.linalg.norm(r_w - r_ref)) / lmin
    return max(floor * float(np.abs(ref.w).max()), bound), r_w
