/*
 * mag_oracle.c -- CPU reference for the weighting equation of metric magnitude.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity oracle: a plain, slow,
 * obviously correct FP64 implementation of what the HIP library computes.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no code, header, table or constant with the HIP path.
 *
 * Arithmetic is written so that every operation rounds as written: build
 * with -ffp-contract=off and without -ffast-math.  OpenMP only distributes
 * independent rows; it never reorders a sum.
 *
 * What it computes (paper, Section 2 "Weightings, magnitude, and diversity"):
 *   d_jk = ||x_j - x_k||_2 over points x_j in R^m              (Section 2)
 *   Z    = exp[-t d], componentwise, t in (0, inf)             (Section 2)
 *   w    : Z w = 1  (eq. weighting); unique since Z is positive definite
 *          for Euclidean d                                     (Section 2)
 *   Mag  = 1^T w                                               (Section 2)
 *   bound t_+ <= log(n-1) / min_{j != k} d_jk                  (Sections 1, 2)
 * and, derived from eq. weighting by differentiating Z(t, X) w = 1:
 *   dw        = -Z^{-1} (dZ) w
 *   dL/dt     = lambda^T (D o Z) w,      lambda = Z^{-1} (gM 1 + gw)
 *   dL/dx_j   = t sum_{k != j} (lambda_j w_k + lambda_k w_j) Z_jk (x_j - x_k) / d_jk
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Euclidean distance between rows j and k of the row-major n x m array X.
 * Exact coordinate differences, summed over l in ascending order. */
static double dist(const double *X, int m, int64_t j, int64_t k)
{
    double s = 0.0;
    for (int l = 0; l < m; ++l) {
        double e = X[j * m + l] - X[k * m + l];
        s = s + e * e;
    }
    return sqrt(s);
}

/* Z_jk = exp(-t d_jk); Z_jj = exp(0) = 1. */
static double zentry(const double *X, int m, double t, int64_t j, int64_t k)
{
    if (j == k)
        return 1.0;
    return exp(-(t * dist(X, m, j, k)));
}

double orc_dist(const double *X, int64_t n, int m, int64_t j, int64_t k)
{
    (void)n;
    return dist(X, m, j, k);
}

/* Full n x n row-major distance matrix. */
void orc_distance_matrix(const double *X, int64_t n, int m, double *D)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t k = 0; k < n; ++k)
            D[j * n + k] = (j == k) ? 0.0 : dist(X, m, j, k);
}

/* Full n x n row-major similarity matrix Z = exp[-t d]. */
void orc_zmatrix(const double *X, int64_t n, int m, double t, double *Z)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t k = 0; k < n; ++k)
            Z[j * n + k] = zentry(X, m, t, j, k);
}

/* min_{j != k} d_jk by brute force over all pairs (bound on t_+). */
double orc_dmin(const double *X, int64_t n, int m)
{
    double best = INFINITY;
#pragma omp parallel for schedule(dynamic, 16) reduction(min : best)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t k = j + 1; k < n; ++k) {
            double d = dist(X, m, j, k);
            if (d < best)
                best = d;
        }
    return best;
}

/* Cholesky factorisation A = L L^T of a symmetric positive definite matrix,
 * computed column by column (the gaxpy / Cholesky-Crout form):
 *   L_jj = sqrt(A_jj - sum_{k<j} L_jk^2)
 *   L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj,   i > j.
 * A is n x n row-major; L overwrites the lower triangle (the strict upper
 * triangle is left untouched and never read).  Returns 0, or j+1 when the
 * j-th pivot is not positive (A not numerically positive definite). */
int orc_cholesky(double *A, int64_t n)
{
    for (int64_t j = 0; j < n; ++j) {
        const double *Lj = A + j * n;
        double s = A[j * n + j];
        for (int64_t k = 0; k < j; ++k)
            s = s - Lj[k] * Lj[k];
        if (!(s > 0.0))
            return (int)(j + 1);
        double ljj = sqrt(s);
        A[j * n + j] = ljj;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            const double *Li = A + i * n;
            double a = Li[j];
            for (int64_t k = 0; k < j; ++k)
                a = a - Li[k] * Lj[k];
            A[i * n + j] = a / ljj;
        }
    }
    return ORC_OK;
}

/* Solve L L^T x = b with the lower factor from orc_cholesky.
 * Forward substitution L y = b row by row, then back substitution
 * L^T x = y column by column (row i of L scatters x_i into y_k, k < i). */
void orc_chol_solve(const double *L, int64_t n, const double *b, double *x)
{
    double *y = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        const double *Li = L + i * n;
        double a = b[i];
        for (int64_t k = 0; k < i; ++k)
            a = a - Li[k] * y[k];
        y[i] = a / Li[i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        const double *Li = L + i * n;
        double xi = y[i] / Li[i];
        x[i] = xi;
        for (int64_t k = 0; k < i; ++k)
            y[k] = y[k] - Li[k] * xi;
    }
    free(y);
}

/* Error-free transformations (Knuth TwoSum; TwoProduct through fma). */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* Residual r_j = 1 - sum_k Z_jk w_k with Z regenerated from X, accumulated
 * by the compensated dot product Dot2 of Ogita, Rump and Oishi (2005): the
 * result is as accurate as if computed in twice the working precision and
 * then rounded.  rows == NULL means all n rows; otherwise r[i] is the
 * residual of row rows[i]. */
void orc_residual(const double *X, int64_t n, int m, double t, const double *w,
                  const int64_t *rows, int64_t nrows, double *r)
{
    int64_t cnt = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t j = rows ? rows[i] : i;
        double s = 1.0, c = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double p, ep, q;
            two_prod(zentry(X, m, t, j, k), -w[k], &p, &ep);
            two_sum(s, p, &s, &q);
            c = c + (q + ep);
        }
        r[i] = s + c;
    }
}

/* Residual r_j = b_j - sum_k Z_jk x_k for a general right-hand side b, by the
 * same Dot2 accumulation as orc_residual (the sum starts from b_j, which is
 * exact).  Used for the solves Z x = b of the gradient (b = gM 1 + gw) and of
 * dw/dt (b = (D o Z) w).  rows == NULL means all n rows. */
void orc_residual_rhs(const double *X, int64_t n, int m, double t, const double *b, const double *x,
                      const int64_t *rows, int64_t nrows, double *r)
{
    int64_t cnt = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t j = rows ? rows[i] : i;
        double s = b[j], c = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double p, ep, q;
            two_prod(zentry(X, m, t, j, k), -x[k], &p, &ep);
            two_sum(s, p, &s, &q);
            c = c + (q + ep);
        }
        r[i] = s + c;
    }
}

/* Plain matrix-vector products with Z regenerated from X, ascending k. */
void orc_zmatvec(const double *X, int64_t n, int m, double t, const double *v, double *y)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t k = 0; k < n; ++k)
            s = s + zentry(X, m, t, j, k) * v[k];
        y[j] = s;
    }
}

/* y = (D o Z) v with (D o Z)_jk = d_jk exp(-t d_jk) (= -dZ_jk/dt). */
void orc_dzmatvec(const double *X, int64_t n, int m, double t, const double *v, double *y)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            if (k == j)
                continue;
            double d = dist(X, m, j, k);
            s = s + d * exp(-(t * d)) * v[k];
        }
        y[j] = s;
    }
}

/* dL/dx_j = t sum_{k != j} (lambda_j w_k + lambda_k w_j) Z_jk (x_j - x_k) / d_jk,
 * written into the row-major n x m array dX. */
void orc_grad_x(const double *X, int64_t n, int m, double t, const double *lam,
                const double *w, double *dX)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t j = 0; j < n; ++j) {
        for (int l = 0; l < m; ++l)
            dX[j * m + l] = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            if (k == j)
                continue;
            double d = dist(X, m, j, k);
            double coef = t * (lam[j] * w[k] + lam[k] * w[j]) * exp(-(t * d)) / d;
            for (int l = 0; l < m; ++l)
                dX[j * m + l] = dX[j * m + l] + coef * (X[j * m + l] - X[k * m + l]);
        }
    }
}

/* The same gradient for selected rows only: dX_rows[i*m + l] = dL/dx_{rows[i], l}.
 * Lets full-size results be checked one output row at a time. */
void orc_grad_x_rows(const double *X, int64_t n, int m, double t, const double *lam,
                     const double *w, const int64_t *rows, int64_t nrows, double *dX_rows)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nrows; ++i) {
        const int64_t j = rows[i];
        for (int l = 0; l < m; ++l)
            dX_rows[i * m + l] = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            if (k == j)
                continue;
            double d = dist(X, m, j, k);
            double coef = t * (lam[j] * w[k] + lam[k] * w[j]) * exp(-(t * d)) / d;
            for (int l = 0; l < m; ++l)
                dX_rows[i * m + l] = dX_rows[i * m + l] + coef * (X[j * m + l] - X[k * m + l]);
        }
    }
}

/* Neumaier's compensated sum (for Mag = 1^T w). */
double orc_sum(const double *v, int64_t n)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double x = v[i];
        double u = s + x;
        if (fabs(s) >= fabs(x))
            c = c + ((s - u) + x);
        else
            c = c + ((x - u) + s);
        s = u;
    }
    return s + c;
}

/* Solve Z x = b given the lower Cholesky factor L of Z (row-major lower
 * triangle of an n x n array; the strict upper triangle is never read):
 * x = L^{-T} L^{-1} b, then `refine` steps x <- x + L^{-T} L^{-1} r with the
 * Dot2 residual r = b - Z x (Z regenerated from X).  b == NULL means the ones
 * vector of eq. weighting.  x_plain (may be NULL) receives the unrefined x. */
void orc_solve_refine(const double *X, int64_t n, int m, double t, const double *L, const double *b,
                      int refine, double *x_plain, double *x)
{
    double *rhs = (double *)malloc((size_t)n * sizeof(double));
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *dx = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        rhs[i] = b ? b[i] : 1.0;
    orc_chol_solve(L, n, rhs, x);
    if (x_plain)
        memcpy(x_plain, x, (size_t)n * sizeof(double));
    for (int it = 0; it < refine; ++it) {
        orc_residual_rhs(X, n, m, t, rhs, x, NULL, 0, r);
        orc_chol_solve(L, n, r, dx);
        for (int64_t i = 0; i < n; ++i)
            x[i] = x[i] + dx[i];
    }
    free(rhs);
    free(r);
    free(dx);
}

/* Weighting by a dense FP64 solve of Z w = 1 (eq. weighting):
 *   1. Z from X (work, n x n row-major), 2. Z = L L^T in place,
 *   3. w_plain = L^{-T} L^{-1} 1,
 *   4. `refine` steps of w <- w + L^{-T} L^{-1} r with r = 1 - Z w from
 *      orc_residual (Dot2), so that w carries no more than unit-roundoff
 *      error for well-conditioned Z.
 * On return `work` holds L (lower triangle).  w_plain may be NULL.
 * Returns 0, or the 1-based index of the failing pivot. */
int orc_weighting(const double *X, int64_t n, int m, double t, int refine,
                  double *w_plain, double *w, double *work)
{
    orc_zmatrix(X, n, m, t, work);
    int st = orc_cholesky(work, n);
    if (st != ORC_OK)
        return st;
    double *ones = (double *)malloc((size_t)n * sizeof(double));
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *dw = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        ones[i] = 1.0;
    orc_chol_solve(work, n, ones, w);
    if (w_plain)
        memcpy(w_plain, w, (size_t)n * sizeof(double));
    for (int it = 0; it < refine; ++it) {
        orc_residual(X, n, m, t, w, NULL, 0, r);
        orc_chol_solve(work, n, r, dw);
        for (int64_t i = 0; i < n; ++i)
            w[i] = w[i] + dw[i];
    }
    free(ones);
    free(r);
    free(dw);
    return ORC_OK;
}

/* ---- weighting at scale zero (Appendix C.1, eq. scaleZero) ---------------
 * As t -> 0, Z(t)^{-1} 1 tends to d^{-1} 1 / (1^T d^{-1} 1).  The distance
 * matrix d is symmetric but indefinite, so the plain solver is Gaussian
 * elimination with partial pivoting. */

/* LU factorisation with row interchanges, in place: P A = L U with unit lower
 * L (strictly below the diagonal) and U (on and above it).  A is n x n
 * row-major; piv[j] is the row swapped with row j at step j.  Returns 0, or
 * j+1 when column j has no nonzero pivot (A singular). */
int orc_lu(double *A, int64_t n, int64_t *piv)
{
    for (int64_t j = 0; j < n; ++j) {
        int64_t p = j;
        double best = fabs(A[j * n + j]);
        for (int64_t i = j + 1; i < n; ++i) {
            double a = fabs(A[i * n + j]);
            if (a > best) {
                best = a;
                p = i;
            }
        }
        piv[j] = p;
        if (!(best > 0.0))
            return (int)(j + 1);
        if (p != j) {
            for (int64_t k = 0; k < n; ++k) {
                double tmp = A[j * n + k];
                A[j * n + k] = A[p * n + k];
                A[p * n + k] = tmp;
            }
        }
        const double ujj = A[j * n + j];
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            double l = A[i * n + j] / ujj;
            A[i * n + j] = l;
            for (int64_t k = j + 1; k < n; ++k)
                A[i * n + k] = A[i * n + k] - l * A[j * n + k];
        }
    }
    return ORC_OK;
}

/* Solve A x = b with the factors of orc_lu: apply the row interchanges to b,
 * forward substitution with unit L, back substitution with U. */
void orc_lu_solve(const double *LU, int64_t n, const int64_t *piv, const double *b, double *x)
{
    for (int64_t i = 0; i < n; ++i)
        x[i] = b[i];
    for (int64_t j = 0; j < n; ++j) {
        if (piv[j] != j) {
            double tmp = x[j];
            x[j] = x[piv[j]];
            x[piv[j]] = tmp;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        double a = x[i];
        for (int64_t k = 0; k < i; ++k)
            a = a - LU[i * n + k] * x[k];
        x[i] = a;
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double a = x[i];
        for (int64_t k = i + 1; k < n; ++k)
            a = a - LU[i * n + k] * x[k];
        x[i] = a / LU[i * n + i];
    }
}

/* Residual r_j = 1 - sum_k d_jk u_k by Dot2 (as orc_residual, with the
 * distances as entries).  rows == NULL means all n rows. */
void orc_dist_residual(const double *X, int64_t n, int m, const double *u, const int64_t *rows, int64_t nrows,
                       double *r)
{
    int64_t cnt = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t j = rows ? rows[i] : i;
        double s = 1.0, c = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double p, ep, q;
            two_prod(dist(X, m, j, k), -u[k], &p, &ep);
            two_sum(s, p, &s, &q);
            c = c + (q + ep);
        }
        r[i] = s + c;
    }
}

/* u = d^{-1} 1 for n >= 2 distinct points: d from X (work, n x n row-major),
 * LU with partial pivoting, one solve, then `refine` steps u <- u + d^{-1} r with
 * the Dot2 residual r = 1 - d u.  Returns 0, or the failing pivot (1-based). */
int orc_dist_solve_ones(const double *X, int64_t n, int m, int refine, double *u, double *work)
{
    orc_distance_matrix(X, n, m, work);
    int64_t *piv = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int st = orc_lu(work, n, piv);
    if (st != ORC_OK) {
        free(piv);
        return st;
    }
    double *ones = (double *)malloc((size_t)n * sizeof(double));
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *du = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        ones[i] = 1.0;
    orc_lu_solve(work, n, piv, ones, u);
    for (int it = 0; it < refine; ++it) {
        orc_dist_residual(X, n, m, u, NULL, 0, r);
        orc_lu_solve(work, n, piv, r, du);
        for (int64_t i = 0; i < n; ++i)
            u[i] = u[i] + du[i];
    }
    free(piv);
    free(ones);
    free(r);
    free(du);
    return ORC_OK;
}
