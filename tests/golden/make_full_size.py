#!/usr/bin/env python3
"""Write the oracle's expected weightings at the full workload sizes.

Calls only ``oracle`` (the CPU reference) and ``workloads`` (seeded inputs).
For each case it stores w as ``<case>.npy`` (FP64, one entry per point) and a
record in ``index.json``: the scale t, the magnitude M = 1^T w (compensated
sum), min w and its index, kappa_M = |w|^T Z |w| / |M|, the oracle's own Dot2
residual ||1 - Z w||_inf, and estimates of Z's extreme eigenvalues (power
iteration with Z, inverse iteration through the factor) that the tests use
to derive their tolerance on w.

Cases:
  * the Gaussian cloud x ~ N(0, I_3), n = 32768, seed 0, at
    t* = 2^(7/8) m^(-2/3) n^(1/4) (eq. gaussianCutoff), t*/4, t*/2, 2 t*, and
    t_b = log(n - 1)/min d (the bound of Sections 1 and 2);
  * the Z^2 rectangle support, n = 8192, seed 0 (the stand-in for Figure 1's
    lattice set), at t in {1/4, 1/2, 1, 2, 4} t_b.

The oracle's own plain column-by-column Cholesky runs at every size (about
half an hour per scale at n = 32768 on 8 cores; OpenBLAS's dpotrf fails at
that size, n^2 = 2^30 entries, so no library factor stands in).  Run:
    python tests/golden/make_full_size.py [--only gauss|z2] [--scales a,b,...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "full_size")


def cases(only, scales):
    out = []
    if only in (None, "gauss"):
        n, m = 32768, 3
        X = W.gaussian(n, m, seed=0)
        ts = float(W.gaussian_cutoff_estimate(n, m))
        tb = oracle.t_bound(X)
        for name, t in (("tstar", ts), ("t_b", tb), ("tstar_over4", ts / 4), ("tstar_over2", ts / 2),
                        ("tstar_x2", 2 * ts)):
            if scales is None or name in scales:
                out.append((f"gauss_n32768_m3_seed0_{name}", "gaussian(32768, 3, seed=0)", X, t))
    if only in (None, "z2"):
        X = W.z2_rectangles(8192, seed=0)
        tb = oracle.t_bound(X)
        for f in (0.25, 0.5, 1.0, 2.0, 4.0):
            out.append((f"z2rect_n8192_seed0_tb_x{f:g}", "z2_rectangles(8192, seed=0)", X, f * tb))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=["gauss", "z2"], default=None)
    ap.add_argument("--scales", default=None, help="comma-separated subset of the Gaussian scales")
    args = ap.parse_args()
    scales = set(args.scales.split(",")) if args.scales else None
    os.makedirs(OUT, exist_ok=True)
    idx_path = os.path.join(OUT, "index.json")
    index = json.load(open(idx_path)) if os.path.exists(idx_path) else {}
    for key, recipe, X, t in cases(args.only, scales):
        t0 = time.time()
        sol = oracle.weighting(X, t, refine=3)
        r = oracle.residual(X, t, sol.w)
        kM = oracle.kappa_M(sol)
        lmax, lmin, cond = oracle.cond_estimate(sol, iters=30, rtol=1e-4)
        np.save(os.path.join(OUT, key + ".npy"), sol.w)
        index[key] = {
            "inputs": recipe, "n": int(X.shape[0]), "m": int(X.shape[1]), "t": float(t),
            "M": float(sol.M), "min_w": float(sol.min_w), "argmin_w": int(sol.argmin),
            "kappa_M": float(kM), "resid_inf": float(np.abs(r).max()),
            "lambda_max_est": float(lmax), "lambda_min_est": float(lmin), "cond_est": float(cond),
            "w_file": key + ".npy", "refine": 3,
        }
        del sol
        with open(idx_path, "w") as f:
            json.dump(index, f, indent=1, sort_keys=True)
        print(f"{key}: t={t:.6g} M={index[key]['M']:.15g} resid={index[key]['resid_inf']:.2e} "
              f"kappa_M={kM:.4g} cond~{cond:.3g} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
