/*
 * mag.h -- C ABI of libmag: the weighting equation of metric magnitude on
 * one AMD Instinct MI355X (gfx950).
 *
 * Problem (Huntsman et al., "Scalably computing metric magnitude", Section 2):
 * given points x_1..x_n in R^m and a scale t in (0, inf),
 *     d_jk = ||x_j - x_k||_2,   Z = exp[-t d] (componentwise),
 *     the weighting w solves Z w = 1              (eq. weighting),
 *     the magnitude is Mag = 1^T w.
 * Z is symmetric positive definite for distinct Euclidean points, so w is
 * unique.  The cutoff t_+ is the least t with w >= 0 (Section 2, cutoff
 * paragraph), bounded above by log(n-1) / min_{j != k} d_jk.
 *
 * Conventions for every entry point:
 *   - Arrays named X, w, dX and the packed batch arrays are DEVICE pointers
 *     on the context's device; scalars and arrays marked HOST are host
 *     memory.  X is row-major n x m FP64 (point j at X[j*m .. j*m+m-1]).
 *   - The caller owns every array passed in; the library never frees or
 *     retains a caller pointer after a call returns.
 *   - Work is enqueued on the context's stream (mag_set_stream); calls
 *     block only to deliver host outputs and status.  A context is
 *     single-stream and not thread-safe.
 *   - Every function returns MAG_OK (0) or a negative error code; nothing
 *     throws across the ABI.  mag_strerror names a code.
 */
#ifndef MAG_H
#define MAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define MAG_OK        0
#define MAG_EINVAL   (-1)  /* n < 1, m < 1, t <= 0 or non-finite, NULL required pointer */
#define MAG_ENOTPD   (-2)  /* Z not positive definite: duplicate points (d_jk = 0, j != k),
                              or breakdown of the FP64 Cholesky                          */
#define MAG_ENOCONV  (-3)  /* refinement did not reach tol; w holds the best iterate      */
#define MAG_ENOMEM   (-4)  /* workspace does not fit in device memory                     */
#define MAG_EHIP     (-5)  /* HIP runtime or library error                                */
#define MAG_EINTERNAL (-6) /* internal consistency failure                                */

const char *mag_strerror(int code);

/* ---- context ------------------------------------------------------------ */
typedef struct mag_ctx mag_ctx;

/* Create a context on HIP device `device`.  It owns all scratch memory
 * (grown on demand, reused across calls, released by mag_destroy). */
int mag_create(mag_ctx **ctx, int device);
void mag_destroy(mag_ctx *ctx);
/* Cap the device memory this context may hold at `bytes` (0 = no cap, the
 * default unless the environment variable MAG_WORKSPACE_LIMIT holds a byte
 * count, optionally with a K, M or G suffix, when the context is created).
 * A call whose workspace would exceed the cap returns MAG_ENOMEM without
 * allocating; buffers already held are kept.  *held (HOST, may be NULL)
 * receives the bytes held now. */
int mag_set_workspace_limit(mag_ctx *ctx, uint64_t bytes);
int mag_workspace_bytes(const mag_ctx *ctx, uint64_t *held);

/* Bound the waits of the sync-free triangular solves (the preconditioner
 * apply of MAG_FP32_IR and mag_prec_apply, the substitution of MAG_FP64_CHOL
 * and mag_chol64_solve) on this context: a workgroup that has polled `polls`
 * times for the block it needs gives up, the kernel finishes, and the call
 * returns MAG_EINTERNAL.  0 (the default) = 2^26 polls, about a minute, far
 * beyond any wait of a correct launch; a small value forces that error path
 * (tests use it).  The batched solves keep the default.  MAG_EINVAL for polls < 0. */
int mag_set_spin_limit(mag_ctx *ctx, int64_t polls);

/* Enqueue subsequent work on `hip_stream` (a hipStream_t; NULL = the
 * context's own stream, a blocking stream: it is ordered with the device's
 * null stream, so work a caller enqueues there -- e.g. PyTorch's default
 * stream, whose handle is NULL -- and the library's work do not overlap). */
int mag_set_stream(mag_ctx *ctx, void *hip_stream);

/* ---- options and diagnostics --------------------------------------------- */
enum {
    MAG_AUTO = 0,        /* by measured cost: MAG_FP32_IR up to n = 49152 (its FP32      *
                          * factor's n^3/3 flops on MFMA are the cheaper solve there:   *
                          * 0.33-0.38 s against 0.27-0.45 s for HODLR at n = 49152),    *
                          * MAG_HODLR above (max_rank 512, one subspace iteration,      *
                          * GMRES(100), up to 400 inner iterations; 0.43-0.65 s against *
                          * 0.77-0.83 s at n = 65536, 0.8-1.5 s against 2.5-2.6 s at    *
                          * n = 98304, on tori, Gaussian and clustered clouds) when     *
                          * m <= 16; if the HODLR solve does not converge, or m > 16,   *
                          * MAG_FP32_IR when its npad^2 factor fits in 3/4 of the       *
                          * device memory, else MAG_ENOMEM                              */
    MAG_FP64_DENSE = 1,  /* FP64 Z in HBM + rocSOLVER dpotrf/dpotrs (dense comparator)   */
    MAG_FP32_IR = 2,     /* FP32 MFMA Cholesky + FP64 GMRES iterative refinement         */
    MAG_HODLR = 3,       /* HODLR preconditioner + FP64 GMRES (largest sizes, Sec. 3.2): *
                          * points reordered by recursive coordinate bisection, leaf    *
                          * blocks exact, sibling blocks Z(I,J) ~ U_I V_J^T sampled     *
                          * with a Gaussian test matrix; m <= 16                        */
    MAG_FP64_CHOL = 5,   /* FP64 Z in HBM + this library's FP64 MFMA blocked Cholesky    *
                          * (64-column diagonal blocks, 256-column panels in pairs, the  *
                          * trailing updates on v_mfma_f64_16x16x4) + the sync-free     *
                          * substitution with that factor: the plain FP64 dense solve    *
                          * on the matrix cores (Sec. 3.2's direct method), no          *
                          * refinement; the dense comparator beside MAG_FP64_DENSE      */
    MAG_HSS = 4          /* HSS preconditioner with nested bases, factored by ULV, + FP64 *
                          * GMRES (Sec. 3.2's hierarchical solver): the same tree; each *
                          * node's basis spans its whole off-diagonal block row (one    *
                          * Gaussian sample, projected up the tree); level l keeps      *
                          * 8 max_rank 2^{-l/2} + oversample columns rounded up to 64   *
                          * (64..512, at most twice its children's: a block row sees    *
                          * the near field on every side); leaves of at least 64 points *
                          * (n > leaf); m <= 16                                         */
};

typedef struct {
    int32_t solver;        /* MAG_AUTO ...                                                */
    int32_t max_outer;     /* refinement steps (residual evaluations), default 10         */
    int32_t gmres_restart; /* Krylov dimension per refinement step, default 30            */
    int32_t max_gmres;     /* total inner iterations over the whole solve, default 200    */
    double tol;            /* target ||1 - Z w||_inf, default 1e-12                       */
    double inner_tol;      /* relative reduction asked of each inner GMRES, default 1e-10 */
    int32_t leaf;          /* HODLR/HSS largest leaf, 2..256, default 128 (else MAG_EINVAL) */
    int32_t max_rank;      /* HODLR rank of the top level's sibling blocks, default 256;  *
                            * level l samples max_rank 2^{-l/2} + oversample columns,     *
                            * rounded up to a multiple of 64 within [64, 512] and the     *
                            * smaller child's size                                        */
    int32_t oversample;    /* HODLR extra sample columns, default 16                      */
    int32_t profile;       /* 1: time phases with HIP events (adds a sync per phase)      */
    uint64_t seed;         /* HODLR sampling seed                                          */
    int32_t inner_prec;    /* MAG_INNER_FP64 (default): every product with Z in FP64;      *
                            * MAG_INNER_FP32: the products inside GMRES evaluate each      *
                            * entry exp(-t d) in FP32 (sums in FP64; m <= 16, else FP64)   *
                            * and ask at most a 1e-6 reduction of each inner solve; the    *
                            * residuals 1 - Z w that decide convergence stay FP64          */
    int32_t diag;          /* diagnostics of mag_weighting / mag_magnitude, default 0:      *
                            * MAG_DIAG_BACKWARD fills mag_info.backward_err (one more       *
                            * FP64 product Z 1); MAG_DIAG_COND fills mag_info.cond_est      *
                            * (Lanczos on Z and on Z^{-1} through the solve's own           *
                            * preconditioner, to 1e-3 relative; about 10 extra products     *
                            * and 10 extra refinement solves)                              */
    int32_t power_iters;   /* HODLR range finder: subspace iterations after the first      *
                            * sample, each replacing the sample Y_I of Z(I, J) by          *
                            * Z(I, J) Z(J, I) orth(Y_I) (Halko, Martinsson and Tropp,      *
                            * 2011, Sec. 4.5), default 0; 0..4 (else MAG_EINVAL); HSS      *
                            * ignores it                                                   */
    int32_t reserved_;     /* zero                                                        */
} mag_opts;

#define MAG_INNER_FP64 0
#define MAG_INNER_FP32 1
#define MAG_DIAG_BACKWARD 1
#define MAG_DIAG_COND 2

/* Fill *opts with the defaults above. */
void mag_opts_default(mag_opts *opts);

typedef struct {
    int32_t status;        /* return code of the call                                     */
    int32_t outer_iters;   /* residual evaluations                                        */
    int32_t gmres_iters;   /* inner corrections: plain refinement steps + GMRES iterations */
    int32_t shifted;       /* 1 if the FP32 factor was taken of Z + shift*I after breakdown */
    double shift;          /* the diagonal shift used (0 if none)                          */
    double resid_inf;      /* ||1 - Z w||_inf as last evaluated on the device (FP64)       */
    double magnitude;      /* 1^T w                                                        */
    double min_w;          /* min_j w_j                                                    */
    int64_t argmin_w;      /* argmin_j w_j                                                 */
    double ms_tilegen;     /* phase times (profile = 1 only)                              */
    double ms_factor;
    double ms_refine;
    double ms_total;
    double ms_update;      /* summed device time of the trailing-update kernel launches   */
    double flop_update;    /* algorithmic flops of those launches                         */
    int32_t n_update;      /* number of trailing-update launches                          */
    int32_t solver;        /* the solver that ran (MAG_AUTO resolved)                      */
    double backward_err;   /* ||1 - Z w||_inf / (||Z||_inf ||w||_inf + 1), the normwise    *
                            * backward error (MAG_DIAG_BACKWARD; else 0)                   */
    double cond_est;       /* lambda_max(Z) / lambda_min(Z) estimated by Lanczos to 1e-3   *
                            * relative (MAG_DIAG_COND; else 0)                              */
} mag_info;

/* ---- the weighting (eq. weighting) ---------------------------------------- */

/* Solve Z w = 1 for the n points X (device, n x m row-major FP64) at scale t;
 * write w (device, n FP64).  opts may be NULL (defaults); info may be NULL.
 * MAG_FP32_IR: w meets ||1 - Z w||_inf <= tol with Z evaluated in FP64, or
 * MAG_ENOCONV is returned with the best iterate in w.  Duplicate points give
 * MAG_ENOTPD.  n = 1 gives w = 1. */
int mag_weighting(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t,
                  double *w, const mag_opts *opts, mag_info *info);

/* As mag_weighting, and return Mag = 1^T w in *M (HOST).  w may be NULL. */
int mag_magnitude(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t,
                  double *M, double *w, const mag_opts *opts, mag_info *info);

/* min_{j != k} ||x_j - x_k|| by brute force over all pairs into *d_min (HOST);
 * the bound on the cutoff is log(n-1)/d_min (Sections 1 and 2).  n >= 2. */
int mag_dmin(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double *d_min);

/* ---- the cutoff t_+ (Section 2, cutoff paragraph and footnote) -------------
 * t_+ is the least t from which w >= 0 (read as inf{t : w(s) >= 0 for all
 * s >= t}).  Search: d_min by brute force gives the bound
 * t_b = log(n-1)/d_min, where w >= 0; a log grid of `grid` points on
 * [t_b*lo_factor, t_b] is scanned downward to the first t with min w < 0
 * (extended downward by lo_factor up to max_extend times); the bracketing
 * cell is then refined in log t by bisection, safeguarded Newton steps using
 * d(min w)/dt = (Z^{-1} (D o Z) w)_{argmin} when newton != 0, until
 * (t_hi - t_lo)/t_hi <= rtol, or until 0 <= min w < eps (eps = 0 means
 * n * 2^-53).  The returned t_plus is the upper end, where min w >= 0.
 * t_lo/t_hi > 0 give a starting bracket (resume); it is verified first. */
typedef struct {
    int32_t grid;          /* grid points, default 32                                     */
    int32_t max_extend;    /* downward grid extensions, default 2                          */
    int32_t newton;        /* 1: safeguarded Newton inside bisection, default 1            */
    int32_t method;        /* bracket refinement: MAG_TPLUS_BISECT (default) or RIDDERS    */
    double lo_factor;      /* grid spans [t_b*lo_factor, t_b], default 1e-3                */
    double rtol;           /* relative bracket width, default 1e-6                         */
    double eps;            /* early halt when 0 <= min w < eps; 0 = n * 2^-53              */
    double t_lo, t_hi;     /* optional starting bracket (0 = none)                          */
} mag_tplus_opts;

/* Ridders' method (Section 2 names it for t_+): in s = log t, with the bracket
 * s_a < s_b (g(s) = min w(e^s), g_a < 0 <= g_b) and g_m at the midpoint s_m, the
 * next point is s_m + (s_m - s_a) sign(g_a - g_b) g_m / sqrt(g_m^2 - g_a g_b),
 * which lies inside the bracket; each step evaluates the midpoint and that point
 * (two solves) and keeps the uppermost sign change among the four.  No
 * derivative is used (newton is ignored). */
#define MAG_TPLUS_BISECT 0
#define MAG_TPLUS_RIDDERS 1

typedef struct {
    double t_plus;         /* = *t_plus                                                     */
    double t_bound;        /* log(n-1)/d_min                                                */
    double d_min;
    double min_w;          /* min w at t_plus                                               */
    double t_bracket_lo, t_bracket_hi;
    int32_t solves;        /* weighting solves (factorisations)                             */
    int32_t newton_steps;  /* interpolated points: Newton (bisection method) or Ridders     */
    int32_t no_sign_change;/* 1: w >= 0 on the whole (extended) grid; t_plus = 0            */
    int32_t status;
} mag_tplus_info;

void mag_tplus_opts_default(mag_tplus_opts *opts);

/* Cutoff search for the points X (device, n x m).  *t_plus (HOST) receives
 * t_+ (0 when no sign change is found: collinear sets and n <= 2 have w > 0
 * for every t).  w (device, n, may be NULL) receives w(t_plus).  topts and
 * sopts (solver options of each weighting solve) may be NULL. */
int mag_tplus(mag_ctx *ctx, const double *X, int64_t n, int32_t m, const mag_tplus_opts *topts,
              const mag_opts *sopts, double *t_plus, double *w, mag_tplus_info *info);

/* dw/dt = Z^{-1} (D o Z) w at scale t, where (D o Z)_jk = d_jk exp(-t d_jk)
 * (from differentiating eq. weighting in t).  w (device, n, may be NULL)
 * receives the weighting, dwdt (device, n) its derivative.  Any m. */
int mag_dwdt(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t, double *w,
             double *dwdt, const mag_opts *opts);

/* ---- weighting at scale zero -------------------------------------------------
 * Appendix C.1 (eq. scaleZero): as t -> 0, Z(t)^{-1} 1 tends to
 *   w0 = d^{-1} 1 / (1^T d^{-1} 1),
 * the solution of d w = 1 scaled to sum 1.  d is indefinite (one positive
 * eigenvalue; -d is positive definite on the complement of 1), so the solve
 * works on B = c 1 1^T - d.  For every c that keeps B nonsingular, B^{-1} 1 =
 * d^{-1} 1 / (c 1^T d^{-1} 1 - 1) (Sherman-Morrison), hence w0 = B^{-1} 1 / (1^T
 * B^{-1} 1) and 1^T d^{-1} 1 = beta / (c beta - 1) with beta = 1^T B^{-1} 1; B is
 * positive definite once c exceeds 1 / (1^T d^{-1} 1).  c starts at twice the
 * largest distance from the centroid (at least the diameter) and is doubled
 * once if the FP32 factor meets a non-positive pivot; the factor's diagonal
 * shift then takes over.  The solve is the FP32_IR path with B in the place of
 * Z (FP32 MFMA Cholesky of B, FP64 refinement with matrix-free products of B,
 * entries c - d_jk).  X: device n x m, distinct points, m <= 16; w: device n.
 * n = 1 gives w0 = 1 (the limit) and 1^T d^{-1} 1 = +inf.  info (may be NULL):
 * iterations, resid_inf = ||1 - B u||_inf of the unscaled solve u, magnitude =
 * the sum of w0, min_w and argmin_w of w0, shifted/shift of the factor.
 * sum_dinv (HOST, may be NULL) receives 1^T d^{-1} 1; c_used (HOST, may be
 * NULL) the c of the solve. */
int mag_weighting_zero(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double *w,
                       const mag_opts *opts, mag_info *info, double *sum_dinv, double *c_used);

/* ---- extreme eigenvalues of Z (positive-definiteness check) ---------------
 * Section 4.2 checks that Z is positive definite, at little cost beside the
 * solve, by estimating its smallest eigenvalue with symmetric Lanczos.  Here:
 *   lambda_max: Lanczos on Z, with the matrix-free FP64 product Z v;
 *   lambda_min: Lanczos on Z^{-1}, each product an FP32-factor + FP64
 *               refinement solve (the factor is computed once, as for
 *               mag_weighting; solver AUTO or FP32_IR, tol from opts);
 * both with full reorthogonalisation (two classical Gram-Schmidt passes).
 * The Ritz value of step j is the extreme eigenvalue of the j x j tridiagonal
 * (bisection on Sturm counts), and r_j = beta_j |s_j| (s: the last entry of its
 * unit eigenvector) bounds the residual of its Ritz vector, so some eigenvalue
 * of the operator lies within r_j of it.  A side stops when r_j <= rtol times
 * its Ritz value, when beta_j vanishes (an invariant subspace: exact), or after
 * max_iter steps.  In exact arithmetic the Ritz values lie inside the spectrum:
 * lambda_max is approached from below and lambda_min from above. */
typedef struct {
    int32_t max_iter;      /* Lanczos steps per side; 0 = 80; at most 256                */
    int32_t pad_;
    double rtol;           /* 0 = 1e-8                                                     */
} mag_eig_opts;

typedef struct {
    double lambda_max, lambda_min, cond;  /* cond = lambda_max / lambda_min               */
    double resid_max;      /* r of the lambda_max side (a bound on Z's residual)           */
    double resid_min;      /* r of the lambda_min side (for Z^{-1}: |1/lambda - mu| <= r)  */
    int32_t iters_max, iters_min;        /* Lanczos steps taken                           */
    int32_t converged;     /* bit 0: the lambda_max side met rtol, bit 1: lambda_min side   */
    int32_t solve_steps;   /* refinement steps over all solves with Z                       */
} mag_eig_info;

void mag_eig_opts_default(mag_eig_opts *opts);

/* Extreme eigenvalues of Z(t) for the points X (device, n x m, distinct).
 * v0 (device, n, may be NULL) starts both sides; NULL uses
 * v0_j = 1/2 + frac((j + 1) g), g = (sqrt(5) - 1)/2, j = 0..n-1.  info (HOST) is
 * required.  MAG_EINVAL for a zero v0 or bad arguments, MAG_ENOTPD for
 * coincident points, MAG_ENOMEM when the FP32 factor does not fit, and the
 * refinement's code when a solve fails (MAG_ENOCONV keeps the values so far). */
int mag_eig_extremes(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t, const double *v0,
                     const mag_eig_opts *eopts, const mag_opts *opts, mag_eig_info *info);

/* ---- adjoint of (w, Mag) with respect to (X, t) ----------------------------
 * Differentiating Z(t, X) w = 1: with lambda = Z^{-1}(gM 1 + gw),
 *   dL/dt   = lambda^T (D o Z) w,
 *   dL/dx_j = t sum_{k != j} (lambda_j w_k + lambda_k w_j) Z_jk (x_j - x_k)/d_jk.
 * mag_weighting_fwd solves like mag_weighting and keeps the FP32 factor in a
 * handle (npad^2 * 4 bytes of device memory, owned by the handle until
 * mag_factor_free); mag_weighting_vjp reuses it for lambda (one refinement
 * solve; none when gw == NULL, since then lambda = gM w). */
typedef struct mag_factor mag_factor;

int mag_weighting_fwd(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t, double *w,
                      mag_factor **keep, const mag_opts *opts, mag_info *info);

/* gM: dL/dMag; gw: dL/dw (device, n, may be NULL); dX: device n x m row-major
 * output (may be NULL); dt: HOST output (may be NULL).  X, n, m, t must be
 * those of the forward call (EINVAL otherwise).  Any m. */
int mag_weighting_vjp(mag_ctx *ctx, mag_factor *f, const double *X, int64_t n, int32_t m,
                      double t, const double *w, double gM, const double *gw, double *dX,
                      double *dt, const mag_opts *opts);

void mag_factor_free(mag_factor *f);

/* ---- batches of problems of uneven n --------------------------------------
 * B problems (clouds and scales) solved together: every phase of the solve is
 * one launch over all problems (device work lists map blocks to problems).  A
 * whole step -- each cloud's next scale, tile generation, factorisation,
 * refinement, min w, bracket update and Newton derivative -- is captured once
 * as a hipGraph and replayed; the refinement and search decisions are taken
 * on the device (a flag word per problem gates every launch), and the host
 * reads one count per step to know when every cloud is done.  The graph holds
 * a plain round and three rounds that may run GMRES(12) cycles; items that
 * mag_weighting_batch finds short of tol after them get the host-driven
 * refinement with the caller's limits.  X packs the clouds row-wise (device);
 * offs (HOST, B+1) gives the row ranges, cloud b = rows [offs[b], offs[b+1]);
 * rows may be shared (several scales of one cloud).  Every item gives the
 * same result as the single call up to rounding order. */

/* w (device, packed like X, rows offs[b]-offs[0] ...) receives each weighting,
 * M (HOST, B, may be NULL) each magnitude, info (HOST, B, may be NULL) each
 * record.  t: HOST, B scales.  Returns MAG_ENOCONV if any item did not meet
 * tol (its info says which). */
int mag_weighting_batch(mag_ctx *ctx, int32_t B, const double *X, const int64_t *offs, int32_t m,
                        const double *t, double *w, double *M, const mag_opts *opts,
                        mag_info *info);

/* Cutoff search of mag_tplus for every cloud, the clouds' grid scans and
 * bracket refinements stepped together.  t_plus (HOST, B) receives each
 * cutoff (0 when no sign change); w (device, packed, may be NULL) the
 * weighting at each cutoff; info (HOST, B, may be NULL). */
int mag_tplus_batch(mag_ctx *ctx, int32_t B, const double *X, const int64_t *offs, int32_t m,
                    const mag_tplus_opts *topts, const mag_opts *sopts, double *t_plus, double *w,
                    mag_tplus_info *info);

/* ---- tuning ----------------------------------------------------------------
 * The single-solve FP32 factor works in panels of 512 columns (256 is the
 * alternative: shorter serial panel work, shallower trailing updates).  The
 * choice is kept on the context per size bucket: the smallest b with
 * npad <= 2^b. */

/* Set the panel width (256 or 512; 0 restores the built-in 512) for the size
 * bucket of n.  MAG_EINVAL for other widths or n < 1. */
int mag_tune_panel(mag_ctx *ctx, int64_t n, int32_t nb);

/* Time the FP32 tile generation + factor of this problem (X: device, n x m)
 * with each panel width, best of `reps` runs each (reps < 1 means 1), and keep
 * the faster for n's size bucket.  nb_out (HOST, may be NULL) receives the
 * choice; ms_out (HOST, 2 doubles, may be NULL) the best times for 256 and
 * 512.  Uses the context's factor workspace (npad^2 floats). */
int mag_autotune(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t, int32_t reps,
                 int32_t *nb_out, double *ms_out);

/* The batched factorisation (mag_weighting_batch, mag_tplus_batch) works in
 * 256-column panels, either in pairs (a strip update of the second panel by
 * the first, then one trailing update with K = 512) or singly (one trailing
 * update with K = 256 per panel: more launches, shallower updates).  The
 * choice is kept per size bucket of the batch's largest npad.
 * mag_tune_batch_group sets it (group 1 single, 2 pairs, 0 the built-in
 * pairs) for the bucket of max_n; MAG_EINVAL for other groups or max_n < 1. */
int mag_tune_batch_group(mag_ctx *ctx, int64_t max_n, int32_t group);

/* Time the batched tile generation + factorisation of these problems (X, offs,
 * m, t as for mag_weighting_batch; every cloud at least one point) with each
 * grouping, best of `reps` graph replays each, and keep the faster for the
 * bucket of the largest npad.  group_out (HOST, may be NULL) receives 1 or 2;
 * ms_out (HOST, 2 doubles, may be NULL) the best times of single panels and
 * pairs.  Uses the context's batch workspace. */
int mag_autotune_batch(mag_ctx *ctx, int32_t B, const double *X, const int64_t *offs, int32_t m,
                       const double *t, int32_t reps, int32_t *group_out, double *ms_out);

/* Write the tuned tables to a JSON text file
 * ({"panel": {"<bucket>": nb, ...}, "batch_group": {"<bucket>": group, ...}}),
 * or read one written by mag_tune_save into the context (entries not in the
 * file are left as they are; "batch_group" may be absent).  MAG_EINVAL on I/O
 * or format errors. */
int mag_tune_save(const mag_ctx *ctx, const char *path);
int mag_tune_load(mag_ctx *ctx, const char *path);

/* ---- kernel-level entry points --------------------------------------------
 * The steps of the FP32_IR path exposed one by one, for parity tests and
 * profiling.  npad = mag_padded_size(n) = n rounded up to a multiple of 256.
 * The FP32 factor layout is column-major with leading dimension npad; rows
 * and columns >= n hold an identity padding. */

/* npad for n points (0 for n < 1). */
int64_t mag_padded_size(int64_t n);

/* y = Z v in FP64 with Z regenerated from X (matrix-free).  v, y: device, n. */
int mag_zmatvec(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t,
                const double *v, double *y);

/* r = 1 - Z w in FP64 (device, n) and *rinf = ||r||_inf (HOST, may be NULL). */
int mag_residual(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t,
                 const double *w, double *r, double *rinf);

/* FP32 Z (tile generator output) into A: device, npad x npad column-major;
 * only the lower triangle and the 128 x 128 diagonal tiles are written. */
int mag_tile32(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t, float *A);

/* FP32 Cholesky factor of Z + shift*I into L (device, npad x npad, lower
 * triangle valid) and the inverses of its 128 x 128 diagonal blocks into dinv
 * (device, npad/128 blocks of 128 x 128 column-major).  *breakdown (HOST, may
 * be NULL) receives 0, or 1 + the index of the first non-positive pivot. */
int mag_factor32(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t,
                 double shift, float *L, float *dinv, int32_t *breakdown);

/* z = (L L^T)^{-1} r with the factor from mag_factor32, FP64 arithmetic;
 * r, z: device, n.  Each call forms the substitution's near tiles
 * (D_b L(b, b-1) and D_b^T L^T(b, b+1) per 128-block, npad * 256 floats of
 * context workspace) from L and dinv, then runs the two triangular solves. */
int mag_prec_apply(mag_ctx *ctx, const float *L, const float *dinv, int64_t n,
                   const double *r, double *z);

/* FP64 Cholesky factor of Z (the MAG_FP64_CHOL factor) into L (device, npad x
 * npad FP64 column-major: L in the lower triangle and L^T in the upper one,
 * identity padding) and the inverses of its 64 x 64 diagonal blocks into dinv
 * (device, npad/64 blocks of 64 x 64 column-major).  *breakdown (HOST, may be
 * NULL) receives 0, or 1 + the index of the first non-positive pivot. */
int mag_factor64(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t,
                 double *L, double *dinv, int32_t *breakdown);

/* z = (L L^T)^{-1} r with the factor from mag_factor64; r, z: device, n. */
int mag_chol64_solve(mag_ctx *ctx, const double *L, const double *dinv, int64_t n,
                     const double *r, double *z);

/* y = (D o Z) v in FP64, matrix-free (device, n); any m. */
int mag_dzmatvec(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t,
                 const double *v, double *y);

/* ---- no-allocation entry point ---------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residual of mag_residual, r = 1 - Z w (device, n) and *rinf = ||r||_inf
 * (HOST, may be NULL), with Z regenerated in FP64 from X (device, n x m, any
 * m), computed without allocating anything.  Its only workspace is a
 * file-scope device array of mag_residual_noalloc_max_doubles() doubles
 * (16 MiB) that each GPU the library runs on holds until the process ends;
 * a call needs npad (1 + s) + npad/256 + 8 of them (s <= 64 column splits,
 * s = 1 from n = 524288 on), so n up to about one million points; larger n
 * returns MAG_ENOMEM without launching anything.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (several streams or
 * threads) race.  The sums run in another order than mag_residual's, so the
 * two agree to the rounding of an n-term FP64 sum, not bitwise. */
int mag_residual_noalloc(mag_ctx *ctx, const double *X, int64_t n, int32_t m, double t,
                         const double *w, double *r, double *rinf);
size_t mag_residual_noalloc_max_doubles(void);

#ifdef __cplusplus
}
#endif

#endif /* MAG_H */
