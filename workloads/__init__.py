"""Seeded synthetic point clouds for the weighting equation Z w = 1.

This module only draws coordinates.  It holds none of the method's arithmetic
(no distances, no similarity matrix, no solve): both the CPU oracle and the
HIP library receive the arrays built here, so they see identical FP64 bits.

Every generator uses numpy's PCG64 (``numpy.random.default_rng(seed)``).

Workloads (the paper measures only synthetic Gaussian clouds, Section 4.3;
its Figure 1 support over Z^2 is not given, so ``z2_rectangles`` stands in):

* ``uniform_square``   n points i.i.d. uniform in [0,1]^2.
* ``z2_rectangles``    unique lattice points of Z^2 drawn with replacement
                       from a random union of axis-aligned rectangles in a
                       200x200 grid (stand-in for the Figure 1 support).
* ``gaussian``         n points from N(0, I_m) or N(0, diag(s)) (Section 4.3).
* ``gaussian_mixture`` mixture of isotropic Gaussians in [0,1]^m.
* ``mixture_clouds``   many mixture clouds of uneven size (batched t_+ search).
* ``noisy_torus``      area-uniform points on a torus plus Gaussian noise.
* ``collinear``        points on a random line in R^m (closed-form fixture).
* ``centre_kgon``      centre plus regular k-gon of unit circumradius.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_square", "z2_rectangles", "gaussian", "gaussian_mixture",
    "mixture_clouds", "noisy_torus", "collinear", "centre_kgon",
    "gaussian_cutoff_estimate", "pack_clouds",
]


def uniform_square(n: int, seed: int = 0, m: int = 2) -> np.ndarray:
    """n points i.i.d. uniform in [0,1]^m, FP64, row-major (n, m)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.random((n, m)), dtype=np.float64)


def z2_rectangles(n: int = 8192, seed: int = 0, n_rect: int = 20,
                  grid: int = 200, draws: int = 12000) -> np.ndarray:
    """Unique points of Z^2 sampled with replacement from a random support.

    The support is the union of ``n_rect`` axis-aligned rectangles, each with
    x-range [min(a,b), max(a,b)] and y-range [min(c,d), max(c,d)], with
    a, b, c, d ~ U{0..grid-1}, inclusive.  ``draws`` cells are drawn uniformly
    with replacement from the support, deduplicated in first-appearance
    order, and the first ``n`` kept; if fewer than ``n`` are unique, further
    batches of 1000 draws are appended.  The nearest-neighbour distance is 1.
    """
    rng = np.random.default_rng(seed)
    mask = np.zeros((grid, grid), dtype=bool)
    for _ in range(n_rect):
        a, b, c, d = rng.integers(0, grid, size=4)
        mask[min(a, b):max(a, b) + 1, min(c, d):max(c, d) + 1] = True
    cells = np.argwhere(mask)  # support, lexicographic order
    if len(cells) < n:
        raise ValueError(f"support has {len(cells)} cells < n={n}")
    seen: dict[tuple[int, int], None] = {}
    batch = draws
    while len(seen) < n:
        idx = rng.integers(0, len(cells), size=batch)
        for i in idx:
            key = (int(cells[i, 0]), int(cells[i, 1]))
            if key not in seen:
                seen[key] = None
                if len(seen) == n:
                    break
        batch = 1000
    pts = np.array(list(seen.keys()), dtype=np.float64)
    return np.ascontiguousarray(pts[:n])


def gaussian(n: int, m: int, seed: int = 0, diag=None) -> np.ndarray:
    """n points from N(0, I_m), or N(0, diag(diag)) when ``diag`` is given."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, m))
    if diag is not None:
        X = X * np.sqrt(np.asarray(diag, dtype=np.float64))[None, :]
    return np.ascontiguousarray(X, dtype=np.float64)


def gaussian_mixture(n: int, m: int = 3, seed: int = 0, k: int = 5,
                     sigma: float = 0.1) -> np.ndarray:
    """Mixture of ``k`` isotropic Gaussians (std ``sigma``) with centres
    uniform in [0,1]^m and equal-weight labels."""
    rng = np.random.default_rng(seed)
    centres = rng.random((k, m))
    labels = rng.integers(0, k, size=n)
    X = centres[labels] + sigma * rng.standard_normal((n, m))
    return np.ascontiguousarray(X, dtype=np.float64)


def mixture_clouds(B: int = 64, m: int = 3, seed: int = 0, n_lo: int = 1000,
                   n_hi: int = 6000, k: int = 5, sigma: float = 0.1):
    """``B`` mixture clouds with sizes n_i ~ U{n_lo..n_hi}; cloud i uses seed
    ``seed + i`` for its points.  Returns a list of (n_i, m) arrays."""
    rng = np.random.default_rng(seed + 1_000_003)
    sizes = rng.integers(n_lo, n_hi + 1, size=B)
    return [gaussian_mixture(int(s), m, seed + i, k, sigma) for i, s in enumerate(sizes)]


def pack_clouds(clouds):
    """Concatenate clouds row-wise; return (X_packed, offsets[B+1] int64)."""
    offs = np.zeros(len(clouds) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(c) for c in clouds])
    X = np.ascontiguousarray(np.concatenate(clouds, axis=0), dtype=np.float64)
    return X, offs


def noisy_torus(n: int, seed: int = 0, R: float = 1.0, r: float = 0.3,
                sigma: float = 0.01) -> np.ndarray:
    """Area-uniform points on a torus (major radius R, minor r) plus
    N(0, sigma^2 I_3) noise.  phi ~ U[0, 2pi); theta drawn by rejection with
    density proportional to R + r cos(theta)."""
    rng = np.random.default_rng(seed)
    phi = rng.random(n) * 2.0 * np.pi
    theta = np.empty(n)
    filled = 0
    while filled < n:
        th = rng.random(2 * (n - filled) + 16) * 2.0 * np.pi
        u = rng.random(th.size) * (R + r)
        keep = th[u <= R + r * np.cos(th)]
        take = min(len(keep), n - filled)
        theta[filled:filled + take] = keep[:take]
        filled += take
    ring = R + r * np.cos(theta)
    X = np.stack([ring * np.cos(phi), ring * np.sin(phi), r * np.sin(theta)], axis=1)
    X = X + sigma * rng.standard_normal((n, 3))
    return np.ascontiguousarray(X, dtype=np.float64)


def collinear(n: int, m: int = 3, seed: int = 0, spread: float = 1.0) -> np.ndarray:
    """n distinct points on a random line through a random origin in R^m.
    Positions along the line are sorted uniform draws (duplicates removed by
    construction with a tiny minimum gap)."""
    rng = np.random.default_rng(seed)
    s = np.sort(rng.random(n)) * spread
    s = s + np.arange(n) * 1e-6 * spread  # strictly increasing
    direction = rng.standard_normal(m)
    direction /= np.linalg.norm(direction)
    origin = rng.standard_normal(m)
    X = origin[None, :] + s[:, None] * direction[None, :]
    return np.ascontiguousarray(X, dtype=np.float64)


def centre_kgon(k: int, m: int = 2) -> np.ndarray:
    """Centre point at the origin plus a regular k-gon of unit circumradius
    in the first two coordinates (remaining coordinates zero)."""
    X = np.zeros((k + 1, m), dtype=np.float64)
    ang = 2.0 * np.pi * np.arange(k) / k
    X[1:, 0] = np.cos(ang)
    X[1:, 1] = np.sin(ang)
    return X


def regular_polygon(k: int, m: int = 2) -> np.ndarray:
    """The vertices of a regular k-gon of unit circumradius in the first two
    coordinates (remaining coordinates zero), in angular order."""
    X = np.zeros((k, m), dtype=np.float64)
    ang = 2.0 * np.pi * np.arange(k) / k
    X[:, 0] = np.cos(ang)
    X[:, 1] = np.sin(ang)
    return X


def gaussian_cutoff_estimate(n: int, m: int) -> float:
    """Empirical law for the cutoff of Gaussian clouds, E t_+ ~ gamma m^(-2/3)
    n^(1/4) with gamma = 2^(7/8) (Appendix C.2, eq. gaussianCutoff).  Used only
    to pick the scale t of the Gaussian benchmark workload."""
    return 2.0 ** (7.0 / 8.0) * m ** (-2.0 / 3.0) * n ** 0.25
