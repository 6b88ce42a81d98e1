// api.hip -- the C ABI of libmag and the solver drivers behind it.
//
// mag_weighting (MAG_FP32_IR) follows the method's three precisions:
//   * the factor Z ~ L L^T is computed in FP32 on MFMA (chol32.hip);
//   * the refinement residual r = 1 - Z w is evaluated in FP64 with Z
//     regenerated from the coordinates (gemv64.hip), and w is updated in FP64;
//   * each correction solves Z d = r by GMRES on the left-preconditioned
//     system (L L^T)^{-1} Z d = (L L^T)^{-1} r, FP64 Krylov vectors and
//     Arnoldi, with the preconditioner applied by FP64 triangular solves that
//     read the FP32 factor (trsv.hip) -- GMRES-based iterative refinement.
// MAG_FP64_DENSE is the dense comparator: FP64 Z in HBM, rocSOLVER
// dpotrf + dpotrs.
#include "internal.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <functional>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

namespace mag {


size_t ctx_held_bytes(const mag_ctx *c)
{
    size_t sum = 0;
    for (const DevBuf *b : {&c->factor, &c->dinv, &c->vecs, &c->partial, &c->ints, &c->aux, &c->bfactor,
                            &c->bdinv, &c->bvec, &c->bscal, &c->bpartial, &c->bints, &c->bdesc, &c->barena,
                            &c->bstage, &c->hodlr, &c->eig, &c->hss})
        sum += b->bytes;
    return sum;
}

int ctx_may_allocate(const mag_ctx *c, size_t extra)
{
    if (c->ws_limit == 0) return MAG_OK;
    return ctx_held_bytes(c) + extra <= c->ws_limit ? MAG_OK : MAG_ENOMEM;
}

int ensure(mag_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes <= b.bytes) return MAG_OK;
    // the cap counts the buffer at its new size in place of its old one
    if (ctx->ws_limit && ctx_held_bytes(ctx) - b.bytes + bytes > ctx->ws_limit) return MAG_ENOMEM;
    if (b.p) {
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) return MAG_EHIP;
        hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return MAG_ENOMEM;
    }
    b.bytes = want;
    return MAG_OK;
}

}  // namespace mag

using namespace mag;

#define HIPCHK0(x)                                  \
    do {                                            \
        if ((x) != hipSuccess) return MAG_EHIP;     \
    } while (0)
#define CHK0(x)                                     \
    do {                                            \
        int rc_ = (x);                              \
        if (rc_ != MAG_OK) return rc_;              \
    } while (0)

namespace mag {
// Polls of one wait of the sync-free substitutions on this context.
long spin_limit_of(const mag_ctx *ctx)
{
    return ctx->spin_limit > 0 ? (long)ctx->spin_limit : kSpinLimitDefault;
}

// Validate the coordinates: finite, and no duplicate points (Z would be
// singular).  One host sync.
int check_points(mag_ctx *ctx, const double *X, int64_t n, int m, bool pairs)
{
    int *status = (int *)ctx->ints.p;
    CHK0(ensure(ctx, ctx->partial, sizeof(double) * std::max<size_t>(dmin_partial_doubles(n) + 8, 64)));
    double *partial = (double *)ctx->partial.p;
    launch_fill_ints(ctx->stream, status, 8, 0);
    launch_check_finite(ctx->stream, X, n * (int64_t)m, status);
    double *dmin2 = partial + dmin_partial_doubles(n);
    pairs = pairs && n >= 2;
    if (pairs) launch_dmin2(ctx->stream, X, n, m, partial, nullptr, dmin2);
    HIPCHK0(hipMemcpyAsync(ctx->host_scalars, status, 8 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    if (pairs)
        HIPCHK0(hipMemcpyAsync(ctx->host_scalars + 8, dmin2, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK0(hipStreamSynchronize(ctx->stream));
    const int *hs = (const int *)ctx->host_scalars;
    if (hs[kStNonFinite]) return MAG_EINVAL;
    if (pairs && !(ctx->host_scalars[8] > 0.0)) return MAG_ENOTPD;
    return MAG_OK;
}

}  // namespace mag


#define HIPCHK(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) return MAG_EHIP;     \
    } while (0)
#define CHK(x)                                      \
    do {                                            \
        int rc_ = (x);                              \
        if (rc_ != MAG_OK) return rc_;              \
    } while (0)

namespace {

constexpr int kIntStatus = 0;    // 8 ints of status
constexpr int kIntCounters = 64;  // preconditioner counters (prec_counter_ints())
constexpr int kIntsTotal = 2048;

struct Timer {
    bool on = false;
    hipStream_t s = nullptr;
    hipEvent_t e[8] = {};
    void start(bool enable, hipStream_t st)
    {
        on = enable;
        s = st;
        if (!on) return;
        for (auto &x : e) hipEventCreate(&x);
    }
    void mark(int i)
    {
        if (on) hipEventRecord(e[i], s);
    }
    double ms(int a, int b)
    {
        if (!on) return 0.0;
        float f = 0.f;
        hipEventSynchronize(e[b]);
        hipEventElapsedTime(&f, e[a], e[b]);
        return f;
    }
    ~Timer()
    {
        if (on)
            for (auto &x : e) hipEventDestroy(x);
    }
};

bool valid_args(const double *X, int64_t n, int32_t m, double t)
{
    return X != nullptr && n >= 1 && m >= 1 && std::isfinite(t) && t > 0.0;
}

int ensure_common(mag_ctx *ctx, int64_t n, int restart)
{
    CHK(ensure(ctx, ctx->ints, sizeof(int) * kIntsTotal));
    const int64_t npad = round_up(n, kPad);
    size_t part = std::max(zmv_partial_doubles(n), blas1_partial_doubles(restart + 2));
    part = std::max(part, dmin_partial_doubles(n) + 8);
    CHK(ensure(ctx, ctx->partial, sizeof(double) * (part + 64)));
    (void)npad;
    return MAG_OK;
}

struct Gmres {
    int restart;
    std::vector<double> H;  // (restart+1) x restart, column-major
    std::vector<double> cs, sn, g;
};

// FP32 factor of Z (+ shift I) with its diagonal-block inverses.
struct Factor32 {
    float *A = nullptr;
    float *dinv = nullptr;
    float *nq = nullptr;  // the substitution's near tiles (launch_near_q, near_q_floats(npad))
    int64_t npad = 0;
    double shift = 0.0;
    int shifted = 0;
};

// Work vectors carved from ctx->vecs (FP64, npad each) and device scalars.
struct Vecs {
    double *V, *x, *r, *z, *ytmp, *u, *best, *rhs, *dsc, *hdev;
};

int carve_vecs(mag_ctx *ctx, int64_t npad, int restart, Vecs &v)
{
    const int nvec = restart + 1 + 7;
    // tail: 16 scalars, then the Hessenberg column staging of 2 (restart + 1) + 1 doubles
    const size_t tail = 16 + 2 * ((size_t)restart + 2) + 64;
    CHK(ensure(ctx, ctx->vecs, sizeof(double) * ((size_t)nvec * npad + tail)));
    double *p = (double *)ctx->vecs.p;
    v.V = p;
    p += (size_t)(restart + 1) * npad;
    v.x = p; p += npad;
    v.r = p; p += npad;
    v.z = p; p += npad;
    v.ytmp = p; p += npad;
    v.u = p; p += npad;
    v.best = p; p += npad;
    v.rhs = p; p += npad;
    v.dsc = p;        // 16 device scalars
    v.hdev = p + 16;  // up to 2*(restart+1)+2 doubles
    return MAG_OK;
}

int ensure_solver(mag_ctx *ctx, int64_t n, int m, int restart)
{
    CHK(ensure_common(ctx, n, restart));
    size_t part = std::max(zmv_partial_doubles(n), pair_partial_doubles(n, m));
    part = std::max(part, blas1_partial_doubles(restart + 2));
    part = std::max(part, dmin_partial_doubles(n) + 8);
    CHK(ensure(ctx, ctx->partial, sizeof(double) * (part + 64)));
    return MAG_OK;
}

// Tile generation + blocked FP32 Cholesky, retried with a growing diagonal
// shift when the FP32 factorisation meets a non-positive pivot.
int factor_fp32(mag_ctx *ctx, const double *X, int64_t n, int m, double t, Factor32 &F,
                FactorTimer *ft, Timer *tm, int kernel = kKernExp)
{
    hipStream_t s = ctx->stream;
    int *status = (int *)ctx->ints.p + kIntStatus;
    double *hs = ctx->host_scalars;
    F.shift = 0.0;
    F.shifted = 0;
    for (int attempt = 0;; ++attempt) {
        launch_fill_ints(s, status, 8, 0);
        // the tile generator also flags coincident points (Z singular)
        launch_tilegen32(s, X, n, m, t, F.A, F.npad, (float)F.shift, status, kernel);
        if (tm && attempt == 0) tm->mark(1);
        if (ft) {
            ft->used = 0;
            ft->flops.clear();
        }
        chol32_factor(s, F.A, F.npad, n, F.dinv, status, ft, panel_width(ctx, F.npad));
        HIPCHK(hipMemcpyAsync(hs, status, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (((const int *)hs)[kStDuplicate]) return MAG_ENOTPD;
        if (((const int *)hs)[kStBreakdown] == 0) break;
        if (attempt >= 6) return MAG_ENOTPD;
        F.shift = (F.shift == 0.0) ? 1e-6 * std::max<double>(1.0, std::sqrt((double)n)) : F.shift * 10.0;
        F.shifted = 1;
    }
    launch_near_q(s, F.A, F.npad, F.dinv, F.nq);
    return MAG_OK;
}

struct RefineStats {
    int outer = 0, inner = 0;
    double resid = INFINITY;
};

// Solve Z x = b (b: device npad vector, zero padded; NULL means the ones
// vector of eq. weighting) by GMRES-based iterative refinement: FP64
// residuals b - Z x with Z regenerated from X, corrections from GMRES on the
// left-preconditioned system (L L^T)^{-1} Z d = (L L^T)^{-1} r.  The best
// iterate goes to xout (device npad).  Stops when ||b - Z x||_inf <= tol *
// max(1, ||b||_inf), on stagnation, or at the iteration limits.
// prec(in, out, tmp): out = M^{-1} in for device npad vectors (tmp: npad scratch)
using PrecFn = std::function<void(const double *, double *, double *)>;

int refine_core(mag_ctx *ctx, const double *X, int64_t n, int m, double t, int64_t npad,
                const PrecFn &prec, const double *b, double bnorm, double *xout, const mag_opts &o,
                RefineStats &st, int kernel = kKernExp)
{
    hipStream_t s = ctx->stream;
    const int restart = std::max(1, o.gmres_restart);
    Vecs v;
    CHK(carve_vecs(ctx, npad, restart, v));
    double *partial = (double *)ctx->partial.p;
    int *ints = (int *)ctx->ints.p;
    int *status = ints + kIntStatus;
    double *hs = ctx->host_scalars;
    const double tol = (o.tol > 0 ? o.tol : 1e-12) * std::max(1.0, bnorm);
    // FP32 entries in the inner products: the correction equation is then solved
    // for an operator within ~1e-7 of Z, so asking GMRES for more than 1e-6 is wasted
    const bool f32_inner = o.inner_prec == MAG_INNER_FP32 && m <= 16 && kernel == kKernExp;
    const double inner_tol = std::max(o.inner_tol > 0 ? o.inner_tol : 1e-10, f32_inner ? 1e-6 : 0.0);
    const int max_gmres = o.max_gmres > 0 ? o.max_gmres : 200;

    const double *bb = b;
    if (!bb) {
        launch_fill(s, v.rhs, npad, 0.0);
        launch_fill(s, v.rhs, n, 1.0);
        bb = v.rhs;
    }
    // x0 = M^{-1} b
    prec(bb, v.x, v.ytmp);

    Gmres G;
    G.restart = restart;
    G.H.assign((size_t)(restart + 1) * restart, 0.0);
    G.cs.assign(restart, 0.0);
    G.sn.assign(restart, 0.0);
    G.g.assign(restart + 1, 0.0);
    std::vector<double> hbuf(2 * (restart + 2) + 2);
    double rnorm = INFINITY, best_norm = INFINITY;
    int rc = MAG_ENOCONV;
    int outer = 0, inner_total = 0;
    // Corrections start as plain refinement steps x += M^{-1} r, which gain
    // about -log10(cond(M^{-1} Z) - 1) digits each when the factor is accurate
    // for this Z; as soon as one gains less than two digits (or none), the
    // iteration restarts from the best iterate with GMRES corrections.
    bool plain = true, last_plain = false;
    auto residual = [&]() -> int {
        launch_zmv(s, X, n, m, t, v.x, v.r, bb, 1, partial, v.dsc, false, kernel);
        HIPCHK(hipMemcpyAsync(hs, v.dsc, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hs + 8, status, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (((const int *)(hs + 8))[kStSpinTimeout]) return MAG_EINTERNAL;
        return MAG_OK;
    };
    for (outer = 0; outer < std::max(1, o.max_outer); ++outer) {
        CHK(residual());
        const double prev = rnorm;
        rnorm = hs[0];
        bool reverted = false;
        if (!(rnorm < best_norm)) {
            if (!last_plain) break;  // no progress: keep the best iterate
            // the plain step did not help: back to the best iterate, GMRES from there
            plain = last_plain = false;
            reverted = true;
            launch_copy(s, v.best, v.x, npad);
            if (++outer >= std::max(1, o.max_outer)) break;
            CHK(residual());
            rnorm = hs[0];
        } else {
            best_norm = rnorm;
            launch_copy(s, v.x, v.best, npad);
        }
        if (rnorm <= tol) {
            rc = MAG_OK;
            break;
        }
        if (last_plain && rnorm > 1e-2 * prev) plain = false;
        else if (!last_plain && !reverted && outer > 0 && rnorm > 0.5 * prev) break;  // stagnation
        if (inner_total >= max_gmres) break;
        if (plain) {
            prec(v.r, v.z, v.ytmp);
            launch_axpy1(s, v.z, v.x, npad);
            ++inner_total;
            last_plain = true;
            continue;
        }
        last_plain = false;
        // GMRES(restart) on M^{-1} Z d = M^{-1} r, d0 = 0
        prec(v.r, v.z, v.ytmp);
        launch_nrm2(s, v.z, npad, partial, v.dsc + 1);
        HIPCHK(hipMemcpyAsync(hs + 1, v.dsc + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double beta = hs[1];
        if (!(beta > 0.0) || !std::isfinite(beta)) break;
        launch_scale_inv(s, v.z, v.V, npad, v.dsc + 1);
        std::fill(G.H.begin(), G.H.end(), 0.0);
        std::fill(G.g.begin(), G.g.end(), 0.0);
        G.g[0] = beta;
        int kdone = 0;
        for (int k = 0; k < restart && inner_total < max_gmres; ++k) {
            double *Vk = v.V + (size_t)k * npad;
            double *Vk1 = v.V + (size_t)(k + 1) * npad;
            launch_zmv(s, X, n, m, t, Vk, v.u, nullptr, 0, partial, nullptr, f32_inner, kernel);
            prec(v.u, Vk1, v.ytmp);
            // classical Gram-Schmidt, twice
            launch_multidot(s, v.V, npad, k + 1, Vk1, npad, partial, v.hdev);
            launch_multi_axpy(s, v.V, npad, k + 1, v.hdev, Vk1, npad, -1.0);
            launch_multidot(s, v.V, npad, k + 1, Vk1, npad, partial, v.hdev + (k + 1));
            launch_multi_axpy(s, v.V, npad, k + 1, v.hdev + (k + 1), Vk1, npad, -1.0);
            launch_nrm2(s, Vk1, npad, partial, v.hdev + 2 * (k + 1));
            HIPCHK(hipMemcpyAsync(hbuf.data(), v.hdev, sizeof(double) * (2 * (k + 1) + 1),
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            const double hk1 = hbuf[2 * (k + 1)];
            double *Hk = G.H.data() + (size_t)k * (restart + 1);
            for (int i = 0; i <= k; ++i) Hk[i] = hbuf[i] + hbuf[k + 1 + i];
            Hk[k + 1] = hk1;
            if (hk1 > 0.0) launch_scale_inv(s, Vk1, Vk1, npad, v.hdev + 2 * (k + 1));
            for (int i = 0; i < k; ++i) {
                const double a = Hk[i], c = Hk[i + 1];
                Hk[i] = G.cs[i] * a + G.sn[i] * c;
                Hk[i + 1] = -G.sn[i] * a + G.cs[i] * c;
            }
            const double a = Hk[k], c = Hk[k + 1];
            const double rr = std::hypot(a, c);
            G.cs[k] = (rr > 0) ? a / rr : 1.0;
            G.sn[k] = (rr > 0) ? c / rr : 0.0;
            Hk[k] = rr;
            Hk[k + 1] = 0.0;
            G.g[k + 1] = -G.sn[k] * G.g[k];
            G.g[k] = G.cs[k] * G.g[k];
            ++inner_total;
            kdone = k + 1;
            if (std::fabs(G.g[k + 1]) <= inner_tol * beta || !(hk1 > 0.0)) break;
        }
        std::vector<double> y(kdone, 0.0);
        for (int i = kdone - 1; i >= 0; --i) {
            double acc = G.g[i];
            for (int j = i + 1; j < kdone; ++j) acc -= G.H[(size_t)j * (restart + 1) + i] * y[j];
            y[i] = acc / G.H[(size_t)i * (restart + 1) + i];
        }
        HIPCHK(hipMemcpyAsync(v.hdev, y.data(), sizeof(double) * kdone, hipMemcpyHostToDevice, s));
        launch_multi_axpy(s, v.V, npad, kdone, v.hdev, v.x, npad, 1.0);
    }
    if (xout != v.best) launch_copy(s, v.best, xout, npad);
    st.outer = outer + (rc == MAG_OK ? 1 : 0);
    st.inner = inner_total;
    st.resid = best_norm;
    return rc;
}

// GMRES-IR with the FP32 Cholesky factor F as the preconditioner (L L^T)^{-1}.
int refine_solve(mag_ctx *ctx, const double *X, int64_t n, int m, double t, const Factor32 &F,
                 const double *b, double bnorm, double *xout, const mag_opts &o, RefineStats &st,
                 int kernel = kKernExp)
{
    int *ints = (int *)ctx->ints.p;
    int *status = ints + kIntStatus;
    int *counters = ints + kIntCounters;
    hipStream_t s = ctx->stream;
    const PrecFn prec = [&](const double *in, double *out, double *tmp) {
        launch_prec_apply(s, F.A, F.npad, F.dinv, in, tmp, out, counters, status, F.nq, spin_limit_of(ctx));
    };
    return refine_core(ctx, X, n, m, t, F.npad, prec, b, bnorm, xout, o, st, kernel);
}

// sum, min, argmin of w[0..n) -> host
int summarize(mag_ctx *ctx, const double *w, int64_t n, double &sum, double &mn, int64_t &am)
{
    hipStream_t s = ctx->stream;
    double *dsc = (double *)ctx->partial.p + blas1_partial_doubles(3);
    launch_sum_min(s, w, n, (double *)ctx->partial.p, dsc);
    HIPCHK(hipMemcpyAsync(ctx->host_scalars + 32, dsc, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    sum = ctx->host_scalars[32];
    mn = ctx->host_scalars[33];
    am = (int64_t)ctx->host_scalars[34];
    return MAG_OK;
}

Factor32 ctx_factor(mag_ctx *ctx, int64_t n)
{
    Factor32 F;
    F.npad = round_up(n, kPad);
    F.A = (float *)ctx->factor.p;
    F.dinv = (float *)ctx->dinv.p;
    F.nq = F.dinv + (size_t)F.npad * kTile;  // ensure_ctx_factor sizes dinv for both
    return F;
}

int ensure_ctx_factor(mag_ctx *ctx, int64_t n)
{
    const int64_t npad = round_up(n, kPad);
    CHK(ensure(ctx, ctx->factor, sizeof(float) * (size_t)npad * (size_t)npad));
    CHK(ensure(ctx, ctx->dinv, sizeof(float) * ((size_t)npad * kTile + near_q_floats(npad))));
    return MAG_OK;
}

using SolveOp = std::function<int(const double *, double *)>;
int ensure_aux(mag_ctx *ctx, int64_t npad);
struct LanczosResult;
int lanczos_top(mag_ctx *ctx, int64_t npad, const SolveOp &op, double *Q, double *u, double *dev, int max_iter,
                double rtol, LanczosResult &res);

// Normwise backward error of the weighting w (device, n):
// ||1 - Z w||_inf / (||Z||_inf ||w||_inf + ||1||_inf), with ||Z||_inf the
// largest entry of Z 1 (every entry of Z is positive) from one FP64 product.
int diag_backward(mag_ctx *ctx, const double *X, int64_t n, int m, double t, const double *w, double rinf,
                  double &eta)
{
    hipStream_t s = ctx->stream;
    const int64_t npad = round_up(n, kPad);
    CHK(ensure_aux(ctx, npad));
    double *aux = (double *)ctx->aux.p;
    double *partial = (double *)ctx->partial.p;
    double *dsc = aux + 4 * npad;
    launch_affine_ones(s, nullptr, 1.0, aux, n, npad);
    launch_zmv(s, X, n, m, t, aux, aux + npad, nullptr, 0, partial, nullptr);
    launch_amax(s, aux + npad, npad, partial, dsc);
    launch_amax(s, w, n, partial, dsc + 1);
    HIPCHK(hipMemcpyAsync(ctx->host_scalars + 48, dsc, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    eta = rinf / (ctx->host_scalars[48] * ctx->host_scalars[49] + 1.0);
    return MAG_OK;
}

// lambda_max(Z) / lambda_min(Z) by Lanczos to relative accuracy 1e-3: on Z
// with matrix-free FP64 products, and on Z^{-1} with `inv` (a solve with the
// caller's preconditioner), from the golden-ratio start vector.
int diag_cond(mag_ctx *ctx, const double *X, int64_t n, int m, double t, const SolveOp &inv, double &cond);

// FP32-factor + FP64 GMRES iterative refinement for Z w = 1, into the
// caller's w (n) -- optionally factorising into caller-provided buffers.
int solve_fp32_ir(mag_ctx *ctx, const double *X, int64_t n, int m, double t, double *w,
                  const mag_opts &o, mag_info *info, Factor32 *keepF = nullptr)
{
    hipStream_t s = ctx->stream;
    const int restart = std::max(1, o.gmres_restart);
    CHK(ensure_solver(ctx, n, m, restart));
    Factor32 F;
    if (keepF) {
        F = *keepF;
    } else {
        CHK(ensure_ctx_factor(ctx, n));
        F = ctx_factor(ctx, n);
    }
    Timer tm;
    tm.start(o.profile != 0, s);
    FactorTimer ft;
    tm.mark(0);
    CHK(factor_fp32(ctx, X, n, m, t, F, o.profile ? &ft : nullptr, &tm));
    if (keepF) *keepF = F;
    tm.mark(2);
    Vecs v;
    CHK(carve_vecs(ctx, F.npad, restart, v));
    RefineStats st;
    int rc = refine_solve(ctx, X, n, m, t, F, nullptr, 1.0, v.best, o, st);
    if (rc != MAG_OK && rc != MAG_ENOCONV) return rc;
    tm.mark(3);
    launch_copy(s, v.best, w, n);
    double sum, mn;
    int64_t am;
    CHK(summarize(ctx, v.best, n, sum, mn, am));
    tm.mark(4);
    if (info) {
        info->outer_iters = st.outer;
        info->gmres_iters = st.inner;
        info->shifted = F.shifted;
        info->shift = F.shift;
        info->resid_inf = st.resid;
        info->magnitude = sum;
        info->min_w = mn;
        info->argmin_w = am;
        if (o.profile) {
            info->ms_tilegen = tm.ms(0, 1);
            info->ms_factor = tm.ms(1, 2);
            info->ms_refine = tm.ms(2, 3);
            info->ms_total = tm.ms(0, 4);
            double msu = 0.0, fl = 0.0;
            for (size_t q = 0; q + 1 < ft.used; q += 2) {
                float f = 0.f;
                hipEventElapsedTime(&f, ft.ev[q], ft.ev[q + 1]);
                msu += f;
                fl += ft.flops[q / 2];
            }
            info->ms_update = msu;
            info->flop_update = fl;
            info->n_update = (int32_t)(ft.used / 2);
        }
        info->solver = MAG_FP32_IR;
        if (o.diag & MAG_DIAG_BACKWARD) CHK(diag_backward(ctx, X, n, m, t, w, st.resid, info->backward_err));
        if (o.diag & MAG_DIAG_COND) {
            mag_opts oi = o;
            oi.tol = 1e-6;
            const SolveOp inv = [&](const double *in, double *out) -> int {
                RefineStats s2;
                const int r2 = refine_solve(ctx, X, n, m, t, F, in, 1.0, out, oi, s2);
                return r2 == MAG_ENOCONV ? MAG_OK : r2;
            };
            CHK(diag_cond(ctx, X, n, m, t, inv, info->cond_est));
        }
    }
    for (auto e : ft.ev) hipEventDestroy(e);
    return rc;
}

int solve_fp64_dense(mag_ctx *ctx, const double *X, int64_t n, int m, double t, double *w,
                     const mag_opts &o, mag_info *info)
{
    hipStream_t s = ctx->stream;
    CHK(ensure_common(ctx, n, 1));
    CHK(ensure(ctx, ctx->factor, sizeof(double) * (size_t)n * (size_t)n));
    CHK(ensure(ctx, ctx->vecs, sizeof(double) * ((size_t)round_up(n, kPad) * 2 + 256)));
    if (!ctx->blas) {
        rocblas_handle h;
        if (rocblas_create_handle(&h) != rocblas_status_success) return MAG_EHIP;
        ctx->blas = h;
    }
    rocblas_handle h = (rocblas_handle)ctx->blas;
    if (rocblas_set_stream(h, s) != rocblas_status_success) return MAG_EHIP;
    double *A = (double *)ctx->factor.p;
    double *r = (double *)ctx->vecs.p;
    double *dsc = r + round_up(n, kPad);
    int *dinfo = (int *)ctx->ints.p + 16;
    double *partial = (double *)ctx->partial.p;
    double *hs = ctx->host_scalars;
    Timer tm;
    tm.start(o.profile != 0, s);
    tm.mark(0);
    launch_tilegen64(s, X, n, m, t, A);
    tm.mark(1);
    if (rocsolver_dpotrf(h, rocblas_fill_lower, (rocblas_int)n, A, (rocblas_int)n, dinfo) !=
        rocblas_status_success)
        return MAG_EHIP;
    tm.mark(2);
    launch_fill(s, w, n, 1.0);
    if (rocsolver_dpotrs(h, rocblas_fill_lower, (rocblas_int)n, 1, A, (rocblas_int)n, w,
                         (rocblas_int)n) != rocblas_status_success)
        return MAG_EHIP;
    tm.mark(3);
    HIPCHK(hipMemcpyAsync(hs + 16, dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*(const int *)(hs + 16) != 0) return MAG_ENOTPD;
    if (info) {
        // diagnostics: residual (FP64 matrix-free) and magnitude
        launch_zmv(s, X, n, m, t, w, r, nullptr, 1, partial, dsc + 4);
        HIPCHK(hipMemcpyAsync(hs + 5, dsc + 4, sizeof(double), hipMemcpyDeviceToHost, s));
        launch_sum_min(s, w, n, partial, dsc);
        HIPCHK(hipMemcpyAsync(hs + 2, dsc, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        info->magnitude = hs[2];
        info->min_w = hs[3];
        info->argmin_w = (int64_t)hs[4];
        info->resid_inf = hs[5];
        info->outer_iters = 0;
        info->gmres_iters = 0;
        if (o.profile) {
            info->ms_tilegen = tm.ms(0, 1);
            info->ms_factor = tm.ms(1, 2);
            info->ms_refine = tm.ms(2, 3);
            info->ms_total = tm.ms(0, 3);
        }
        info->solver = MAG_FP64_DENSE;
        if (o.diag & MAG_DIAG_BACKWARD) CHK(diag_backward(ctx, X, n, m, t, w, info->resid_inf, info->backward_err));
        if (o.diag & MAG_DIAG_COND) {
            const SolveOp inv = [&](const double *in, double *out) -> int {
                HIPCHK(hipMemcpyAsync(out, in, sizeof(double) * round_up(n, kPad), hipMemcpyDeviceToDevice, s));
                if (rocsolver_dpotrs(h, rocblas_fill_lower, (rocblas_int)n, 1, A, (rocblas_int)n, out,
                                     (rocblas_int)n) != rocblas_status_success)
                    return MAG_EHIP;
                return MAG_OK;
            };
            CHK(diag_cond(ctx, X, n, m, t, inv, info->cond_est));
        }
    }
    return MAG_OK;
}


// FP64 Z in HBM in the padded layout + this library's FP64 MFMA blocked
// Cholesky + the sync-free substitution with the FP64 factor: the plain dense
// FP64 solve on the matrix cores (no refinement).
int solve_fp64_chol(mag_ctx *ctx, const double *X, int64_t n, int m, double t, double *w, const mag_opts &o,
                    mag_info *info)
{
    hipStream_t s = ctx->stream;
    const int64_t npad = round_up(n, kPad);
    CHK(ensure_common(ctx, n, 1));
    CHK(ensure(ctx, ctx->factor, sizeof(double) * (size_t)npad * (size_t)npad));
    CHK(ensure(ctx, ctx->dinv, sizeof(double) * (size_t)npad * 64));
    CHK(ensure(ctx, ctx->vecs, sizeof(double) * ((size_t)npad * 3 + 256)));
    double *A = (double *)ctx->factor.p;
    double *dinv = (double *)ctx->dinv.p;
    double *rhs = (double *)ctx->vecs.p;
    double *ytmp = rhs + npad;
    double *z = ytmp + npad;
    double *dsc = z + npad;
    int *ints = (int *)ctx->ints.p;
    int *status = ints + kIntStatus;
    double *partial = (double *)ctx->partial.p;
    double *hs = ctx->host_scalars;
    FactorTimer ft;
    Timer tm;
    tm.start(o.profile != 0, s);
    tm.mark(0);
    launch_fill_ints(s, status, 8, 0);
    launch_tilegen64p(s, X, n, m, t, A, npad, status);
    tm.mark(1);
    chol64_factor(s, A, npad, n, dinv, status, o.profile ? &ft : nullptr);
    tm.mark(2);
    launch_affine_ones(s, nullptr, 1.0, rhs, n, npad);
    launch_chol64_solve(s, A, npad, dinv, rhs, ytmp, z, ints + kIntCounters, status, spin_limit_of(ctx));
    HIPCHK(hipMemcpyAsync(w, z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    tm.mark(3);
    HIPCHK(hipMemcpyAsync(hs + 16, status, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int rc = MAG_OK;
    {
        const int *st = (const int *)(hs + 16);
        if (st[kStSpinTimeout]) rc = MAG_EINTERNAL;
        else if (st[kStDuplicate] || st[kStBreakdown]) rc = MAG_ENOTPD;
    }
    if (rc == MAG_OK && info) {
        // diagnostics: residual (FP64 matrix-free) and magnitude
        launch_zmv(s, X, n, m, t, w, z, nullptr, 1, partial, dsc + 4);
        HIPCHK(hipMemcpyAsync(hs + 5, dsc + 4, sizeof(double), hipMemcpyDeviceToHost, s));
        launch_sum_min(s, w, n, partial, dsc);
        HIPCHK(hipMemcpyAsync(hs + 2, dsc, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        info->magnitude = hs[2];
        info->min_w = hs[3];
        info->argmin_w = (int64_t)hs[4];
        info->resid_inf = hs[5];
        info->outer_iters = 0;
        info->gmres_iters = 0;
        if (o.profile) {
            info->ms_tilegen = tm.ms(0, 1);
            info->ms_factor = tm.ms(1, 2);
            info->ms_refine = tm.ms(2, 3);
            info->ms_total = tm.ms(0, 3);
            double msu = 0.0, fl = 0.0;
            for (size_t q = 0; q + 1 < ft.used; q += 2) {
                float f = 0.f;
                hipEventElapsedTime(&f, ft.ev[q], ft.ev[q + 1]);
                msu += f;
                fl += ft.flops[q / 2];
            }
            info->ms_update = msu;
            info->flop_update = fl;
            info->n_update = (int32_t)(ft.used / 2);
        }
        info->solver = MAG_FP64_CHOL;
        if (o.diag & MAG_DIAG_BACKWARD) CHK(diag_backward(ctx, X, n, m, t, w, info->resid_inf, info->backward_err));
        if (o.diag & MAG_DIAG_COND) {
            const SolveOp inv = [&](const double *in, double *out) -> int {
                // in, out: npad vectors zero in the padding
                launch_chol64_solve(s, A, npad, dinv, in, ytmp, out, ints + kIntCounters, status,
                                    spin_limit_of(ctx));
                return MAG_OK;
            };
            CHK(diag_cond(ctx, X, n, m, t, inv, info->cond_est));
        }
    }
    for (auto e : ft.ev) hipEventDestroy(e);
    return rc;
}


// HODLR preconditioner (hodlr.hip) + FP64 GMRES-IR with matrix-free Z v.
int solve_hodlr(mag_ctx *ctx, const double *X, int64_t n, int m, double t, double *w,
                const mag_opts &o, mag_info *info)
{
    hipStream_t s = ctx->stream;
    const int restart = std::max(1, o.gmres_restart);
    const int leaf = o.leaf > 0 ? o.leaf : hodlr_default_leaf();
    if (leaf < 2 || leaf > hodlr_max_leaf() || m > 16) return MAG_EINVAL;
    CHK(ensure_solver(ctx, n, m, restart));
    Timer tm;
    tm.start(o.profile != 0, s);
    tm.mark(0);
    HodlrFactor H;
    if (o.power_iters < 0 || o.power_iters > 4) return MAG_EINVAL;
    CHK(hodlr_factor(ctx, X, n, m, t, leaf, std::max(0, o.max_rank), std::max(0, o.oversample), o.power_iters,
                     o.seed, H));
    tm.mark(1);
    tm.mark(2);
    Vecs v;
    CHK(carve_vecs(ctx, H.npad, restart, v));
    const PrecFn prec = [&](const double *in, double *out, double *) { hodlr_apply(s, H, in, out); };
    RefineStats st;
    int rc = refine_core(ctx, X, n, m, t, H.npad, prec, nullptr, 1.0, v.best, o, st);
    if (rc != MAG_OK && rc != MAG_ENOCONV) return rc;
    tm.mark(3);
    launch_copy(s, v.best, w, n);
    double sum, mn;
    int64_t am;
    CHK(summarize(ctx, v.best, n, sum, mn, am));
    tm.mark(4);
    if (info) {
        info->outer_iters = st.outer;
        info->gmres_iters = st.inner;
        info->resid_inf = st.resid;
        info->magnitude = sum;
        info->min_w = mn;
        info->argmin_w = am;
        if (o.profile) {
            info->ms_tilegen = 0.0;
            info->ms_factor = tm.ms(0, 1);
            info->ms_refine = tm.ms(2, 3);
            info->ms_total = tm.ms(0, 4);
        }
        info->solver = MAG_HODLR;
        if (o.diag & MAG_DIAG_BACKWARD) CHK(diag_backward(ctx, X, n, m, t, w, st.resid, info->backward_err));
        if (o.diag & MAG_DIAG_COND) {
            mag_opts oi = o;
            oi.tol = 1e-6;
            const SolveOp inv = [&](const double *in, double *out) -> int {
                RefineStats s2;
                const int r2 = refine_core(ctx, X, n, m, t, H.npad, prec, in, 1.0, out, oi, s2);
                return r2 == MAG_ENOCONV ? MAG_OK : r2;
            };
            CHK(diag_cond(ctx, X, n, m, t, inv, info->cond_est));
        }
    }
    return rc;
}

// HSS preconditioner with nested bases + ULV (hodlr.hip) + FP64 GMRES-IR.
int solve_hss(mag_ctx *ctx, const double *X, int64_t n, int m, double t, double *w, const mag_opts &o,
              mag_info *info)
{
    hipStream_t s = ctx->stream;
    const int restart = std::max(1, o.gmres_restart);
    const int leaf = o.leaf > 0 ? o.leaf : hodlr_default_leaf();
    if (leaf < 2 || leaf > hodlr_max_leaf() || m > 16) return MAG_EINVAL;
    CHK(ensure_solver(ctx, n, m, restart));
    Timer tm;
    tm.start(o.profile != 0, s);
    tm.mark(0);
    HssFactor H;
    CHK(hss_factor(ctx, X, n, m, t, leaf, std::max(0, o.max_rank), std::max(0, o.oversample), o.seed, H));
    if (info) {
        info->shifted = H.shift > 0.0 ? 1 : 0;
        info->shift = H.shift;
    }
    tm.mark(1);
    tm.mark(2);
    Vecs v;
    CHK(carve_vecs(ctx, H.npad, restart, v));
    int prc = MAG_OK;
    const PrecFn prec = [&](const double *in, double *out, double *) {
        const int e = hss_apply(s, H, in, out);
        if (e != MAG_OK) prc = e;
    };
    RefineStats st;
    int rc = refine_core(ctx, X, n, m, t, H.npad, prec, nullptr, 1.0, v.best, o, st);
    if (prc != MAG_OK) return prc;
    if (rc != MAG_OK && rc != MAG_ENOCONV) return rc;
    tm.mark(3);
    launch_copy(s, v.best, w, n);
    double sum, mn;
    int64_t am;
    CHK(summarize(ctx, v.best, n, sum, mn, am));
    tm.mark(4);
    if (info) {
        info->outer_iters = st.outer;
        info->gmres_iters = st.inner;
        info->resid_inf = st.resid;
        info->magnitude = sum;
        info->min_w = mn;
        info->argmin_w = am;
        if (o.profile) {
            info->ms_tilegen = 0.0;
            info->ms_factor = tm.ms(0, 1);
            info->ms_refine = tm.ms(2, 3);
            info->ms_total = tm.ms(0, 4);
        }
        info->solver = MAG_HSS;
        if (o.diag & MAG_DIAG_BACKWARD) CHK(diag_backward(ctx, X, n, m, t, w, st.resid, info->backward_err));
        if (o.diag & MAG_DIAG_COND) {
            mag_opts oi = o;
            oi.tol = 1e-6;
            const SolveOp inv = [&](const double *in, double *out) -> int {
                RefineStats s2;
                const int r2 = refine_core(ctx, X, n, m, t, H.npad, prec, in, 1.0, out, oi, s2);
                if (prc != MAG_OK) return prc;
                return r2 == MAG_ENOCONV ? MAG_OK : r2;
            };
            CHK(diag_cond(ctx, X, n, m, t, inv, info->cond_est));
        }
    }
    return rc;
}

// MAG_AUTO takes the HODLR preconditioner above this size.  Measured on the
// MI355X, whole solves (noisy torus at t = 0.5, 2, 8; Gaussian cloud at its
// cutoff scale; mixture of five Gaussians at t = 30, 100): n = 49152: dense
// FP32 factor + refinement 330-376 ms, HODLR 272-455 ms; n = 65536: 767-828 ms
// against 425-647 ms (HODLR with max_rank 512 and one subspace iteration);
// n = 98304: 2.47-2.62 s against 0.82-1.45 s.  The clustered clouds compress
// worst and put the crossover near the upper sizes; without the subspace
// iteration the HODLR solve of the mixture at t = 30 stalls at n = 131072.
constexpr int64_t kAutoHodlrMinN = 49152;

// Whether the dense FP32 factor's npad^2 floats fit in three quarters of the
// device memory (counting what this context already holds for it) and in the
// context's cap.
bool auto_dense(mag_ctx *ctx, int64_t n)
{
    size_t fr = 0, tot = 0;
    const double npad = (double)round_up(n, kPad);
    const double need = 4.0 * npad * npad;
    if (ctx->ws_limit && need > (double)ctx->ws_limit) return false;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return true;
    return need <= 0.75 * ((double)fr + (double)ctx->factor.bytes);
}

// dw/dt = Z^{-1} (D o Z) w with the factor F of Z(t) (differentiating
// eq. weighting in t).  w, out: device npad vectors.  Uses ctx->vecs.
int dwdt_with_factor(mag_ctx *ctx, const double *X, int64_t n, int m, double t, const Factor32 &F,
                     const double *w, double *out, const mag_opts &o, RefineStats &st)
{
    hipStream_t s = ctx->stream;
    double *aux = (double *)ctx->aux.p;  // [0, npad): (D o Z) w
    double *partial = (double *)ctx->partial.p;
    launch_dzmv(s, X, n, m, t, w, aux, partial);
    double *amax = aux + 4 * F.npad;  // scalar slot after the four aux vectors
    launch_amax(s, aux, F.npad, partial, amax);
    HIPCHK(hipMemcpyAsync(ctx->host_scalars + 40, amax, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return refine_solve(ctx, X, n, m, t, F, aux, ctx->host_scalars[40], out, o, st);
}

int ensure_aux(mag_ctx *ctx, int64_t npad)
{
    return ensure(ctx, ctx->aux, sizeof(double) * ((size_t)npad * 4 + 64));
}

// ---- symmetric tridiagonal helpers of the Lanczos estimator (host) ----------
// T: diagonal a[0..k), off-diagonal b[0..k-1).

// Number of eigenvalues of T below x: negative pivots of the LDL^T
// factorisation of T - x I (Sylvester's law of inertia).
int sturm_below(const std::vector<double> &a, const std::vector<double> &b, int k, double x, double tiny)
{
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < k; ++i) {
        q = (a[i] - x) - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
        if (q == 0.0) q = -tiny;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Largest eigenvalue of T by bisection on the Sturm count, started from the
// Gershgorin interval.
double tridiag_top(const std::vector<double> &a, const std::vector<double> &b, int k)
{
    double lo = INFINITY, hi = -INFINITY, scale = 0.0;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
        scale = std::max(scale, std::fabs(a[i]) + r);
    }
    const double tiny = std::max(scale, 1e-300) * 1e-300;
    for (int it = 0; it < 2200 && hi - lo > 2.0 * DBL_EPSILON * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_below(a, b, k, mid, tiny) == k) hi = mid;  // every eigenvalue below mid
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Last entry of the unit eigenvector of T for the eigenvalue theta: inverse
// iteration, (T - theta I) y = z solved by Gaussian elimination with partial
// pivoting on the tridiagonal (row swaps fill a second superdiagonal).
double tridiag_last(const std::vector<double> &a, const std::vector<double> &b, int k, double theta)
{
    if (k == 1) return 1.0;
    double scale = 0.0;
    for (int i = 0; i < k; ++i) scale = std::max(scale, std::fabs(a[i]) + (i + 1 < k ? std::fabs(b[i]) : 0.0));
    const double tiny = DBL_EPSILON * std::max(scale, 1e-300);
    std::vector<double> d(k), dl(k - 1), du(k - 1), du2(k, 0.0);
    std::vector<char> swp(k - 1, 0);
    for (int i = 0; i < k; ++i) d[i] = a[i] - theta;
    for (int i = 0; i + 1 < k; ++i) dl[i] = du[i] = b[i];
    for (int i = 0; i + 1 < k; ++i) {
        if (std::fabs(d[i]) >= std::fabs(dl[i])) {
            if (d[i] == 0.0) d[i] = tiny;
            const double l = dl[i] / d[i];
            dl[i] = l;
            d[i + 1] -= l * du[i];
        } else {
            // rows i and i+1 trade places; the pivot row brings its superdiagonal along
            const double l = d[i] / dl[i];
            d[i] = dl[i];
            dl[i] = l;
            const double u0 = du[i];
            du[i] = d[i + 1];
            d[i + 1] = u0 - l * d[i + 1];
            if (i + 2 < k) {
                du2[i] = du[i + 1];
                du[i + 1] = -l * du[i + 1];
            }
            swp[i] = 1;
        }
    }
    if (d[k - 1] == 0.0) d[k - 1] = tiny;
    std::vector<double> y(k, 1.0 / std::sqrt((double)k));
    for (int it = 0; it < 3; ++it) {
        for (int i = 0; i + 1 < k; ++i) {
            if (swp[i]) {
                const double y0 = y[i];
                y[i] = y[i + 1];
                y[i + 1] = y0 - dl[i] * y[i];
            } else {
                y[i + 1] -= dl[i] * y[i];
            }
        }
        y[k - 1] /= d[k - 1];
        y[k - 2] = (y[k - 2] - du[k - 2] * y[k - 1]) / d[k - 2];
        for (int i = k - 3; i >= 0; --i) y[i] = (y[i] - du[i] * y[i + 1] - du2[i] * y[i + 2]) / d[i];
        double nrm = 0.0;
        for (int i = 0; i < k; ++i) nrm = std::max(nrm, std::fabs(y[i]));
        for (int i = 0; i < k; ++i) y[i] /= nrm;  // keep the scale bounded between steps
    }
    double nrm2 = 0.0;
    for (int i = 0; i < k; ++i) nrm2 += y[i] * y[i];
    return y[k - 1] / std::sqrt(nrm2);
}

struct LanczosResult {
    double theta = 0.0, resid = 0.0;
    int iters = 0;
    bool converged = false;
};

// Symmetric Lanczos for the largest eigenvalue of the operator applied by
// op(in, out) (device npad vectors, zero on the padding), from q0 (device npad,
// unit 2-norm).  Q holds max_iter + 1 basis vectors of npad doubles; u is a
// work vector; dev: 2 * (max_iter + 2) device doubles.  Every new vector is
// orthogonalised against the whole basis twice (classical Gram-Schmidt).
int lanczos_top(mag_ctx *ctx, int64_t npad, const std::function<int(const double *, double *)> &op,
                double *Q, double *u, double *dev, int max_iter, double rtol, LanczosResult &res)
{
    hipStream_t s = ctx->stream;
    double *partial = (double *)ctx->partial.p;
    // the dot products of step j write partial sums for j + 1 vectors
    if (ctx->partial.bytes < sizeof(double) * blas1_partial_doubles(max_iter + 1)) return MAG_EINTERNAL;
    std::vector<double> a, b, hbuf(2 * (max_iter + 2) + 1);
    for (int j = 0; j < max_iter; ++j) {
        double *qj = Q + (size_t)j * npad;
        double *qj1 = Q + (size_t)(j + 1) * npad;
        CHK(op(qj, u));
        launch_multidot(s, Q, npad, j + 1, u, npad, partial, dev);
        launch_multi_axpy(s, Q, npad, j + 1, dev, u, npad, -1.0);
        launch_multidot(s, Q, npad, j + 1, u, npad, partial, dev + (j + 1));
        launch_multi_axpy(s, Q, npad, j + 1, dev + (j + 1), u, npad, -1.0);
        launch_nrm2(s, u, npad, partial, dev + 2 * (j + 1));
        HIPCHK(hipMemcpyAsync(hbuf.data(), dev, sizeof(double) * (2 * (j + 1) + 1), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        a.push_back(hbuf[j] + hbuf[2 * j + 1]);  // q_j . A q_j over both passes
        const double beta = hbuf[2 * (j + 1)];
        const int k = j + 1;
        res.theta = tridiag_top(a, b, k);
        res.iters = k;
        if (!std::isfinite(res.theta) || !std::isfinite(beta)) return MAG_EINTERNAL;
        if (!(beta > 1e-14 * std::fabs(res.theta))) {  // invariant subspace: T's eigenvalues are exact
            res.resid = std::fabs(beta);
            res.converged = true;
            return MAG_OK;
        }
        res.resid = beta * std::fabs(tridiag_last(a, b, k, res.theta));
        if (res.resid <= rtol * std::fabs(res.theta)) {
            res.converged = true;
            return MAG_OK;
        }
        b.push_back(beta);
        if (k < max_iter) launch_scale_inv(s, u, qj1, npad, dev + 2 * (j + 1));
    }
    return MAG_OK;
}

int diag_cond(mag_ctx *ctx, const double *X, int64_t n, int m, double t, const SolveOp &inv, double &cond)
{
    constexpr int kIters = 40;
    constexpr double kRtol = 1e-3;
    hipStream_t s = ctx->stream;
    const int64_t npad = round_up(n, kPad);
    CHK(ensure(ctx, ctx->partial, std::max(ctx->partial.bytes, sizeof(double) * (blas1_partial_doubles(kIters + 2) + 64))));
    CHK(ensure(ctx, ctx->eig, sizeof(double) * ((size_t)(kIters + 3) * npad + 2 * (kIters + 2) + 64)));
    double *Q = (double *)ctx->eig.p;
    double *u = Q + (size_t)(kIters + 1) * npad;
    double *q0 = u + npad;
    double *dev = q0 + npad;
    double *partial = (double *)ctx->partial.p;
    launch_golden(s, q0, n, npad);
    launch_nrm2(s, q0, npad, partial, dev);
    HIPCHK(hipMemcpyAsync(ctx->host_scalars + 50, dev, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double q0norm = ctx->host_scalars[50];
    const SolveOp zop = [&](const double *in, double *out) -> int {
        launch_zmv(s, X, n, m, t, in, out, nullptr, 0, partial, nullptr);
        return MAG_OK;
    };
    LanczosResult top, bot;
    launch_scale(s, q0, 1.0 / q0norm, Q, npad, npad);
    CHK(lanczos_top(ctx, npad, zop, Q, u, dev, kIters, kRtol, top));
    launch_scale(s, q0, 1.0 / q0norm, Q, npad, npad);
    CHK(lanczos_top(ctx, npad, inv, Q, u, dev, kIters, kRtol, bot));
    cond = (bot.theta > 0.0) ? top.theta * bot.theta : INFINITY;
    return MAG_OK;
}

}  // namespace

struct mag_factor {
    int device = 0;
    int64_t n = 0;
    int32_t m = 0;
    double t = 0.0;
    Factor32 F;
};

namespace {

// One weighting solve at scale t for the cutoff search: w into dst (device,
// npad), returns min w and argmin; optionally dw/dt at argmin.
struct TEval {
    double t = 0.0, minw = 0.0, dmin_dt = 0.0;
    int64_t arg = -1;
    bool has_deriv = false;
};

// d(min w)/dt at the point of the last solve, whose factor is still in ctx:
// (dw/dt)_{argmin} with dw/dt = Z^{-1} (D o Z) w.
int tplus_deriv(mag_ctx *ctx, const double *X, int64_t n, int m, const mag_opts &o,
                const double *w, TEval &ev)
{
    Factor32 F = ctx_factor(ctx, n);
    double *d = (double *)ctx->aux.p + 2 * F.npad;
    RefineStats st2;
    int rc2 = dwdt_with_factor(ctx, X, n, m, ev.t, F, w, d, o, st2);
    if (rc2 == MAG_OK || rc2 == MAG_ENOCONV) {
        HIPCHK(hipMemcpyAsync(ctx->host_scalars + 41, d + ev.arg, sizeof(double),
                              hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ev.dmin_dt = ctx->host_scalars[41];
        ev.has_deriv = std::isfinite(ev.dmin_dt);
    } else if (rc2 != MAG_OK) {
        return rc2;
    }
    return MAG_OK;
}

int tplus_eval(mag_ctx *ctx, const double *X, int64_t n, int m, double t, const mag_opts &o,
               bool deriv, double *dst, TEval &ev, int &solves)
{
    const int restart = std::max(1, o.gmres_restart);
    Factor32 F = ctx_factor(ctx, n);
    CHK(factor_fp32(ctx, X, n, m, t, F, nullptr, nullptr));
    RefineStats st;
    int rc = refine_solve(ctx, X, n, m, t, F, nullptr, 1.0, dst, o, st);
    if (rc != MAG_OK && rc != MAG_ENOCONV) return rc;
    ++solves;
    double sum;
    CHK(summarize(ctx, dst, n, sum, ev.minw, ev.arg));
    ev.t = t;
    ev.has_deriv = false;
    (void)restart;
    if (deriv) return tplus_deriv(ctx, X, n, m, o, dst, ev);
    return MAG_OK;
}

}  // namespace

namespace {
// MAG_WORKSPACE_LIMIT: a byte count with an optional K, M or G suffix (powers of
// 1024); unset, empty or unreadable means no cap.
size_t workspace_limit_from_env()
{
    const char *e = std::getenv("MAG_WORKSPACE_LIMIT");
    if (!e || !*e) return 0;
    char *end = nullptr;
    const double v = std::strtod(e, &end);
    if (end == e || !(v > 0.0) || !std::isfinite(v)) return 0;
    double mul = 1.0;
    if (*end == 'K' || *end == 'k') mul = 1024.0;
    else if (*end == 'M' || *end == 'm') mul = 1024.0 * 1024.0;
    else if (*end == 'G' || *end == 'g') mul = 1024.0 * 1024.0 * 1024.0;
    return (size_t)(v * mul);
}
}  // namespace

namespace {
// Parse the object {"<bucket>": value, ...} that follows `key` in text into
// staged/any; values must satisfy ok(v).  MAG_EINVAL on malformed input; a
// missing key leaves everything unset when optional.
template <class Ok>
int parse_bucket_map(const std::string &text, const char *key, bool optional, int (&staged)[64], bool (&any)[64],
                     Ok ok)
{
    const size_t at = text.find(key);
    if (at == std::string::npos) return optional ? MAG_OK : MAG_EINVAL;
    size_t p = text.find('{', at);
    const size_t end = (p == std::string::npos) ? std::string::npos : text.find('}', p);
    if (end == std::string::npos) return MAG_EINVAL;
    while (true) {
        const size_t q0 = text.find('"', p + 1);
        if (q0 == std::string::npos || q0 > end) break;
        const size_t q1 = text.find('"', q0 + 1);
        const size_t colon = (q1 == std::string::npos) ? std::string::npos : text.find(':', q1);
        if (colon == std::string::npos || colon > end) return MAG_EINVAL;
        char *stop = nullptr;
        const long b = std::strtol(text.c_str() + q0 + 1, &stop, 10);
        if (stop != text.c_str() + q1 || b < 0 || b >= 64) return MAG_EINVAL;
        const long v = std::strtol(text.c_str() + colon + 1, &stop, 10);
        if (stop == text.c_str() + colon + 1 || !ok(v)) return MAG_EINVAL;
        staged[b] = (int)v;
        any[b] = true;
        p = (size_t)(stop - text.c_str());
    }
    return MAG_OK;
}
}  // namespace

extern "C" {

const char *mag_strerror(int code)
{
    switch (code) {
    case MAG_OK: return "ok";
    case MAG_EINVAL: return "invalid argument";
    case MAG_ENOTPD: return "similarity matrix not positive definite (duplicate points?)";
    case MAG_ENOCONV: return "refinement did not reach the tolerance";
    case MAG_ENOMEM: return "out of device memory";
    case MAG_EHIP: return "HIP runtime or library error";
    case MAG_EINTERNAL: return "internal error";
    default: return "unknown error";
    }
}

void mag_opts_default(mag_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->solver = MAG_AUTO;
    o->max_outer = 10;
    o->gmres_restart = 30;
    o->max_gmres = 200;
    o->tol = 1e-12;
    o->inner_tol = 1e-10;
    o->leaf = 128;
    o->max_rank = 256;
    o->oversample = 16;
    o->profile = 0;
    o->seed = 0x9E3779B97F4A7C15ull;
    o->inner_prec = MAG_INNER_FP64;
    o->diag = 0;
    o->power_iters = 0;
}

int mag_create(mag_ctx **out, int device)
{
    if (!out) return MAG_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return MAG_EINVAL;
    HIPCHK(hipSetDevice(device));
    mag_ctx *c = new mag_ctx();
    c->device = device;
    // a blocking stream: work on it is ordered with the device's null stream, which
    // is where callers that pass NULL to mag_set_stream (PyTorch's default stream)
    // put their allocations, fills and copies
    if (hipStreamCreateWithFlags(&c->own_stream, hipStreamDefault) != hipSuccess) {
        delete c;
        return MAG_EHIP;
    }
    c->stream = c->own_stream;
    if (hipHostMalloc((void **)&c->host_scalars, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        hipStreamDestroy(c->own_stream);
        delete c;
        return MAG_EHIP;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cu_count = cus;
    c->ws_limit = workspace_limit_from_env();
    if (noalloc_setup(device) != MAG_OK) {
        mag_destroy(c);
        return MAG_EHIP;
    }
    if (ensure(c, c->ints, sizeof(int) * kIntsTotal) != MAG_OK) {
        mag_destroy(c);
        return MAG_ENOMEM;
    }
    *out = c;
    return MAG_OK;
}

void mag_destroy(mag_ctx *c)
{
    if (!c) return;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    for (DevBuf *b : {&c->factor, &c->dinv, &c->vecs, &c->partial, &c->ints, &c->aux, &c->bfactor,
                      &c->bdinv, &c->bvec, &c->bscal, &c->bpartial, &c->bints, &c->bdesc, &c->barena,
                      &c->bstage, &c->hodlr, &c->eig, &c->hss})
        if (b->p) hipFree(b->p);
    if (c->bhost) hipHostFree(c->bhost);
    if (c->blas) rocblas_destroy_handle((rocblas_handle)c->blas);
    if (c->host_scalars) hipHostFree(c->host_scalars);
    if (c->own_stream) hipStreamDestroy(c->own_stream);
    delete c;
}

int mag_set_workspace_limit(mag_ctx *c, uint64_t bytes)
{
    if (!c) return MAG_EINVAL;
    c->ws_limit = (size_t)bytes;
    return MAG_OK;
}

int mag_set_spin_limit(mag_ctx *c, int64_t polls)
{
    if (!c || polls < 0) return MAG_EINVAL;
    c->spin_limit = polls;
    return MAG_OK;
}

int mag_workspace_bytes(const mag_ctx *c, uint64_t *held)
{
    if (!c || !held) return MAG_EINVAL;
    *held = (uint64_t)ctx_held_bytes(c);
    return MAG_OK;
}

int mag_set_stream(mag_ctx *c, void *stream)
{
    if (!c) return MAG_EINVAL;
    c->stream = stream ? (hipStream_t)stream : c->own_stream;
    return MAG_OK;
}

int64_t mag_padded_size(int64_t n) { return n < 1 ? 0 : round_up(n, kPad); }

int mag_tune_panel(mag_ctx *c, int64_t n, int32_t nb)
{
    if (!c || n < 1 || (nb != 0 && nb != 256 && nb != 512)) return MAG_EINVAL;
    c->tune_panel[size_bucket(round_up(n, kPad))] = nb;
    return MAG_OK;
}

int mag_autotune(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, int32_t reps,
                 int32_t *nb_out, double *ms_out)
{
    if (!c || !valid_args(X, n, m, t)) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    CHK(ensure_common(c, n, 1));
    CHK(check_points(c, X, n, m));
    CHK(ensure_ctx_factor(c, n));
    const int64_t npad = round_up(n, kPad);
    hipStream_t s = c->stream;
    float *A = (float *)c->factor.p;
    float *dinv = (float *)c->dinv.p;
    int *status = (int *)c->ints.p + kIntStatus;
    const int widths[2] = {256, 512};
    double best[2] = {INFINITY, INFINITY};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int rc = MAG_OK;
    for (int rep = 0; rep < std::max(1, reps) && rc == MAG_OK; ++rep) {
        for (int q = 0; q < 2; ++q) {
            launch_fill_ints(s, status, 8, 0);
            if (hipEventRecord(e0, s) != hipSuccess) { rc = MAG_EHIP; break; }
            launch_tilegen32(s, X, n, m, t, A, npad, 0.0f);
            chol32_factor(s, A, npad, n, dinv, status, nullptr, widths[q]);
            float ms = 0.0f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = MAG_EHIP;
                break;
            }
            best[q] = std::min(best[q], (double)ms);
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc != MAG_OK) return rc;
    const int pick = (best[0] < best[1]) ? 256 : 512;
    c->tune_panel[size_bucket(npad)] = pick;
    if (nb_out) *nb_out = pick;
    if (ms_out) {
        ms_out[0] = best[0];
        ms_out[1] = best[1];
    }
    return MAG_OK;
}

int mag_tune_save(const mag_ctx *c, const char *path)
{
    if (!c || !path) return MAG_EINVAL;
    FILE *f = std::fopen(path, "w");
    if (!f) return MAG_EINVAL;
    std::fprintf(f, "{\"panel\": {");
    bool first = true;
    for (int b = 0; b < 64; ++b) {
        if (c->tune_panel[b] == 0) continue;
        std::fprintf(f, "%s\"%d\": %d", first ? "" : ", ", b, c->tune_panel[b]);
        first = false;
    }
    std::fprintf(f, "}, \"batch_group\": {");
    first = true;
    for (int b = 0; b < 64; ++b) {
        if (c->tune_bgroup[b] == 0) continue;
        std::fprintf(f, "%s\"%d\": %d", first ? "" : ", ", b, c->tune_bgroup[b]);
        first = false;
    }
    std::fprintf(f, "}}\n");
    return std::fclose(f) == 0 ? MAG_OK : MAG_EINVAL;
}



int mag_tune_load(mag_ctx *c, const char *path)
{
    if (!c || !path) return MAG_EINVAL;
    FILE *f = std::fopen(path, "r");
    if (!f) return MAG_EINVAL;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
    int staged[64] = {}, bstaged[64] = {};
    bool any[64] = {}, bany[64] = {};
    CHK(parse_bucket_map(text, "\"panel\"", false, staged, any,
                         [](long v) { return v == 0 || v == 256 || v == 512; }));
    CHK(parse_bucket_map(text, "\"batch_group\"", true, bstaged, bany, [](long v) { return v >= 0 && v <= 2; }));
    for (int b = 0; b < 64; ++b) {
        if (any[b]) c->tune_panel[b] = staged[b];
        if (bany[b]) c->tune_bgroup[b] = bstaged[b];
    }
    return MAG_OK;
}



int mag_dmin(mag_ctx *c, const double *X, int64_t n, int32_t m, double *d_min)
{
    if (!c || !X || !d_min || n < 2 || m < 1) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    CHK(ensure(c, c->partial, sizeof(double) * (dmin_partial_doubles(n) + 64)));
    double *partial = (double *)c->partial.p;
    double *out = partial + dmin_partial_doubles(n);
    launch_dmin2(c->stream, X, n, m, partial, nullptr, out);
    HIPCHK(hipMemcpyAsync(c->host_scalars, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *d_min = std::sqrt(c->host_scalars[0]);
    return MAG_OK;
}

int mag_weighting(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, double *w,
                  const mag_opts *opts, mag_info *info)
{
    if (info) std::memset(info, 0, sizeof(*info));
    if (!c || !w || !valid_args(X, n, m, t)) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    mag_opts o;
    if (opts) o = *opts;
    else mag_opts_default(&o);
    CHK(ensure_common(c, n, std::max(1, o.gmres_restart)));
    // MAG_AUTO: the HODLR preconditioner above the measured crossover, the dense
    // FP32 factor below it or when the HODLR solve does not converge
    const bool auto_hodlr = o.solver == MAG_AUTO && n > kAutoHodlrMinN && m <= 16;
    // the FP32 path's tile generator checks the pairs itself (no separate O(n^2) pass)
    const bool fp32 = o.solver == MAG_FP32_IR || (o.solver == MAG_AUTO && !auto_hodlr);
    int rc = check_points(c, X, n, m, !fp32);
    if (rc == MAG_OK && n == 1) {
        launch_fill(c->stream, w, 1, 1.0);
        HIPCHK(hipStreamSynchronize(c->stream));
        if (info) {
            info->magnitude = 1.0;
            info->min_w = 1.0;
            info->solver = MAG_FP32_IR;
        }
    } else if (rc == MAG_OK) {
        switch (o.solver) {
        case MAG_FP64_DENSE: rc = solve_fp64_dense(c, X, n, m, t, w, o, info); break;
        case MAG_FP64_CHOL: rc = solve_fp64_chol(c, X, n, m, t, w, o, info); break;
        case MAG_HODLR: rc = solve_hodlr(c, X, n, m, t, w, o, info); break;
        case MAG_HSS: rc = solve_hss(c, X, n, m, t, w, o, info); break;
        case MAG_AUTO:
            if (auto_hodlr) {
                mag_opts oh = o;
                oh.max_rank = std::max(oh.max_rank, 512);
                oh.power_iters = std::max(oh.power_iters, 1);
                oh.gmres_restart = std::max(oh.gmres_restart, 100);
                oh.max_gmres = std::max(oh.max_gmres, 400);
                oh.max_outer = std::max(oh.max_outer, 30);
                CHK(ensure_common(c, n, oh.gmres_restart));
                rc = solve_hodlr(c, X, n, m, t, w, oh, info);
                if (rc == MAG_ENOCONV && auto_dense(c, n)) rc = solve_fp32_ir(c, X, n, m, t, w, o, info);
            } else if (auto_dense(c, n)) {
                rc = solve_fp32_ir(c, X, n, m, t, w, o, info);
            } else {
                rc = MAG_ENOMEM;
            }
            break;
        case MAG_FP32_IR: rc = solve_fp32_ir(c, X, n, m, t, w, o, info); break;
        default: rc = MAG_EINVAL; break;
        }
    }
    if (info) info->status = rc;
    return rc;
}

int mag_magnitude(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, double *M,
                  double *w, const mag_opts *opts, mag_info *info)
{
    if (!c || !M) return MAG_EINVAL;
    mag_info local;
    mag_info *inf = info ? info : &local;
    double *wbuf = w;
    DevBuf tmp;
    if (!wbuf) {
        if (!valid_args(X, n, m, t)) return MAG_EINVAL;
        HIPCHK(hipSetDevice(c->device));
        CHK(ctx_may_allocate(c, sizeof(double) * n));
        if (hipMalloc(&tmp.p, sizeof(double) * n) != hipSuccess) return MAG_ENOMEM;
        wbuf = (double *)tmp.p;
    }
    int rc = mag_weighting(c, X, n, m, t, wbuf, opts, inf);
    if (tmp.p) {
        hipStreamSynchronize(c->stream);
        hipFree(tmp.p);
    }
    if (rc == MAG_OK || rc == MAG_ENOCONV) *M = inf->magnitude;
    return rc;
}


// ---- kernel-level entry points (parity tests, profiling) -------------------

int mag_zmatvec(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, const double *v,
                double *y)
{
    if (!c || !v || !y || !valid_args(X, n, m, t)) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    CHK(ensure_common(c, n, 1));
    const int64_t npad = round_up(n, kPad);
    CHK(ensure(c, c->vecs, sizeof(double) * ((size_t)npad + 256)));
    double *ybuf = (double *)c->vecs.p;
    launch_zmv(c->stream, X, n, m, t, v, ybuf, nullptr, 0, (double *)c->partial.p, nullptr);
    HIPCHK(hipMemcpyAsync(y, ybuf, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return MAG_OK;
}

int mag_residual(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, const double *w,
                 double *r, double *rinf)
{
    if (!c || !w || !r || !valid_args(X, n, m, t)) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    CHK(ensure_common(c, n, 1));
    const int64_t npad = round_up(n, kPad);
    CHK(ensure(c, c->vecs, sizeof(double) * ((size_t)npad + 256)));
    double *rbuf = (double *)c->vecs.p;
    double *dsc = rbuf + npad;
    launch_zmv(c->stream, X, n, m, t, w, rbuf, nullptr, 1, (double *)c->partial.p, dsc);
    HIPCHK(hipMemcpyAsync(r, rbuf, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->host_scalars, dsc, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (rinf) *rinf = c->host_scalars[0];
    return MAG_OK;
}

int mag_tile32(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, float *A)
{
    if (!c || !A || !valid_args(X, n, m, t)) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    launch_tilegen32(c->stream, X, n, m, t, A, round_up(n, kPad), 0.0f);
    HIPCHK(hipStreamSynchronize(c->stream));
    return MAG_OK;
}

int mag_factor32(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, double shift,
                 float *L, float *dinv, int32_t *breakdown)
{
    if (!c || !L || !dinv || !valid_args(X, n, m, t) || !(shift >= 0.0)) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    CHK(ensure(c, c->ints, sizeof(int) * kIntsTotal));
    const int64_t npad = round_up(n, kPad);
    int *status = (int *)c->ints.p;
    launch_fill_ints(c->stream, status, 8, 0);
    launch_tilegen32(c->stream, X, n, m, t, L, npad, (float)shift);
    chol32_factor(c->stream, L, npad, n, dinv, status, nullptr, panel_width(c, npad));
    HIPCHK(hipMemcpyAsync(c->host_scalars, status, 8 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (breakdown) *breakdown = ((const int *)c->host_scalars)[kStBreakdown];
    return MAG_OK;
}

int mag_prec_apply(mag_ctx *c, const float *L, const float *dinv, int64_t n, const double *r,
                   double *z)
{
    if (!c || !L || !dinv || !r || !z || n < 1) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    CHK(ensure(c, c->ints, sizeof(int) * kIntsTotal));
    const int64_t npad = round_up(n, kPad);
    // three vectors, then the substitution's near tiles (formed from L and dinv per call)
    const size_t vec_doubles = (size_t)npad * 3 + 256;
    CHK(ensure(c, c->vecs, sizeof(double) * vec_doubles + sizeof(float) * near_q_floats(npad)));
    double *rb = (double *)c->vecs.p;
    double *yt = rb + npad;
    double *zb = yt + npad;
    float *nq = (float *)(rb + vec_doubles);
    int *ints = (int *)c->ints.p;
    launch_fill_ints(c->stream, ints, 8, 0);
    launch_fill(c->stream, rb, npad, 0.0);
    HIPCHK(hipMemcpyAsync(rb, r, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    launch_near_q(c->stream, L, npad, dinv, nq);
    launch_prec_apply(c->stream, L, npad, dinv, rb, yt, zb, ints + kIntCounters, ints, nq, spin_limit_of(c));
    HIPCHK(hipMemcpyAsync(z, zb, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->host_scalars, ints, 8 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (((const int *)c->host_scalars)[kStSpinTimeout]) return MAG_EINTERNAL;
    return MAG_OK;
}

int mag_factor64(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, double *L, double *dinv,
                 int32_t *breakdown)
{
    if (!c || !L || !dinv || !valid_args(X, n, m, t)) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    CHK(ensure(c, c->ints, sizeof(int) * kIntsTotal));
    const int64_t npad = round_up(n, kPad);
    int *status = (int *)c->ints.p;
    launch_fill_ints(c->stream, status, 8, 0);
    launch_tilegen64p(c->stream, X, n, m, t, L, npad, nullptr);
    chol64_factor(c->stream, L, npad, n, dinv, status, nullptr);
    HIPCHK(hipMemcpyAsync(c->host_scalars, status, 8 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (breakdown) *breakdown = ((const int *)c->host_scalars)[kStBreakdown];
    return MAG_OK;
}

int mag_chol64_solve(mag_ctx *c, const double *L, const double *dinv, int64_t n, const double *r, double *z)
{
    if (!c || !L || !dinv || !r || !z || n < 1) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    CHK(ensure(c, c->ints, sizeof(int) * kIntsTotal));
    const int64_t npad = round_up(n, kPad);
    CHK(ensure(c, c->vecs, sizeof(double) * ((size_t)npad * 3 + 256)));
    double *rb = (double *)c->vecs.p;
    double *yt = rb + npad;
    double *zb = yt + npad;
    int *ints = (int *)c->ints.p;
    launch_fill_ints(c->stream, ints, 8, 0);
    launch_fill(c->stream, rb, npad, 0.0);
    HIPCHK(hipMemcpyAsync(rb, r, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    launch_chol64_solve(c->stream, L, npad, dinv, rb, yt, zb, ints + kIntCounters, ints, spin_limit_of(c));
    HIPCHK(hipMemcpyAsync(z, zb, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->host_scalars, ints, 8 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (((const int *)c->host_scalars)[kStSpinTimeout]) return MAG_EINTERNAL;
    return MAG_OK;
}


// ---- cutoff search ----------------------------------------------------------

void mag_tplus_opts_default(mag_tplus_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->grid = 32;
    o->max_extend = 2;
    o->newton = 1;
    o->lo_factor = 1e-3;
    o->rtol = 1e-6;
    o->eps = 0.0;
}

int mag_tplus(mag_ctx *c, const double *X, int64_t n, int32_t m, const mag_tplus_opts *topts,
              const mag_opts *sopts, double *t_plus, double *w_out, mag_tplus_info *info)
{
    if (info) std::memset(info, 0, sizeof(*info));
    if (!c || !X || !t_plus || n < 1 || m < 1) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    mag_tplus_opts to;
    if (topts) to = *topts;
    else mag_tplus_opts_default(&to);
    mag_opts o;
    if (sopts) o = *sopts;
    else mag_opts_default(&o);
    if (to.grid < 2 || !(to.lo_factor > 0.0 && to.lo_factor < 1.0) || !(to.rtol > 0.0)) return MAG_EINVAL;
    if (to.method != MAG_TPLUS_BISECT && to.method != MAG_TPLUS_RIDDERS) return MAG_EINVAL;
    const int restart = std::max(1, o.gmres_restart);
    CHK(ensure_solver(c, n, m, restart));
    int rc = check_points(c, X, n, m);
    if (rc != MAG_OK) return rc;
    *t_plus = 0.0;
    if (n <= 2) {
        // one or two points: w > 0 for every t (w_j = 1/(1 + e^{-td}))
        if (info) {
            info->no_sign_change = 1;
            info->min_w = n == 1 ? 1.0 : 0.5;
            info->status = MAG_OK;
        }
        return MAG_OK;
    }
    const int64_t npad = round_up(n, kPad);
    CHK(ensure_ctx_factor(c, n));
    CHK(ensure_aux(c, npad));
    double dmin = 0.0;
    CHK(mag_dmin(c, X, n, m, &dmin));
    const double tb = std::log((double)(n - 1)) / dmin;
    const double eps = to.eps > 0.0 ? to.eps : (double)n * std::ldexp(1.0, -53);
    double *w_hi = (double *)c->aux.p + 3 * npad;  // weighting at the current upper end
    double *w_cur = (double *)c->aux.p + npad;
    int solves = 0, newton_steps = 0;
    TEval lo, hi, cur;
    bool have_lo = false, have_hi = false;
    const bool ridders = to.method == MAG_TPLUS_RIDDERS;
    const bool newton = to.newton != 0 && !ridders;

    auto accept_hi = [&](const TEval &e) -> int {
        hi = e;
        have_hi = true;
        launch_copy(c->stream, w_cur, w_hi, npad);
        return MAG_OK;
    };

    // optional caller bracket (resume): verify the signs, else fall back to the grid
    if (to.t_lo > 0.0 && to.t_hi > to.t_lo) {
        CHK(tplus_eval(c, X, n, m, to.t_hi, o, newton, w_cur, cur, solves));
        if (cur.minw >= 0.0) {
            accept_hi(cur);
            CHK(tplus_eval(c, X, n, m, to.t_lo, o, newton, w_cur, cur, solves));
            if (cur.minw < 0.0) {
                lo = cur;
                have_lo = true;
            }
        }
        if (!have_lo) have_hi = false;
    }
    if (!have_lo) {
        // downward scan of a log grid from the bound (readings: largest sign change)
        double top = tb;
        for (int ext = 0; ext <= to.max_extend && !have_lo; ++ext) {
            for (int i = to.grid - 1; i >= 0; --i) {
                const double tt = top * std::pow(to.lo_factor, (double)(to.grid - 1 - i) / (to.grid - 1));
                if (have_hi && tt >= hi.t) continue;
                CHK(tplus_eval(c, X, n, m, tt, o, false, w_cur, cur, solves));
                if (cur.minw < 0.0) {
                    lo = cur;
                    have_lo = true;
                    break;
                }
                accept_hi(cur);
                if (cur.minw < eps && cur.minw >= 0.0 && ext == 0 && i == to.grid - 1) {
                    // w already at the halting threshold at the bound
                }
            }
            top *= to.lo_factor;
        }
    }
    if (!have_lo) {
        if (info) {
            info->no_sign_change = 1;
            info->t_bound = tb;
            info->d_min = dmin;
            info->min_w = have_hi ? hi.minw : 0.0;
            info->solves = solves;
            info->status = MAG_OK;
        }
        return MAG_OK;
    }
    // Ridders' method in log t: each step evaluates the midpoint and then the
    // Ridders point from the bracket values at the step's start; both lie inside
    // the bracket on the root's side, and each update keeps lo < 0 <= hi, the
    // uppermost sign change.
    int guard = 0;
    bool halted = false;
    auto take = [&](const TEval &e) -> int {
        if (e.minw < 0.0) {
            lo = e;
        } else {
            CHK(accept_hi(e));
            if (e.minw < eps) halted = true;  // halting rule: 0 <= min w < eps
        }
        return MAG_OK;
    };
    while (ridders && !halted && (hi.t - lo.t) / hi.t > to.rtol && guard++ < 200) {
        const double sa = std::log(lo.t), sb = std::log(hi.t), ga = lo.minw, gb = hi.minw;
        const double tm = std::exp(0.5 * (sa + sb));
        if (!(tm > lo.t && tm < hi.t)) break;
        CHK(tplus_eval(c, X, n, m, tm, o, false, w_cur, cur, solves));
        CHK(take(cur));
        if (halted || (hi.t - lo.t) / hi.t <= to.rtol) break;
        const double tx = std::exp(ridders_point(sa, ga, sb, gb, cur.minw));
        if (!(tx > lo.t && tx < hi.t)) continue;
        CHK(tplus_eval(c, X, n, m, tx, o, false, w_cur, cur, solves));
        ++newton_steps;
        CHK(take(cur));
    }
    // otherwise refine the bracket [lo, hi]: safeguarded Newton in log t inside
    // bisection.  The last evaluated point is lo, whose factor is still in the
    // context, so its derivative costs one refinement solve rather than a
    // factorisation.
    TEval last = lo;
    if (newton) {
        CHK(tplus_deriv(c, X, n, m, o, w_cur, last));
        lo = last;
    }
    bool prev_newton = false;
    double prev_step = INFINITY;
    while (!ridders && (hi.t - lo.t) / hi.t > to.rtol && guard++ < 200) {
        const double slo = std::log(lo.t), shi = std::log(hi.t);
        const double mid = 0.5 * (slo + shi);
        double sc = mid;
        bool use_newton = false;
        if (newton && last.has_deriv && last.dmin_dt != 0.0) {
            // g(s) = min w(e^s), g'(s) = t * d(min w)/dt
            const double sl = std::log(last.t);
            const double sn = sl - last.minw / (last.t * last.dmin_dt);
            const double step = std::fabs(sn - sl);
            if (sn > slo && sn < shi && (!prev_newton || step <= 0.5 * prev_step)) {
                sc = sn;
                use_newton = true;
                prev_step = step;
                // next to a bracket end: step just past the predicted root so
                // that the bracket closes to rtol
                const double close = 0.25 * to.rtol;
                if (sc - slo < close) sc = std::min(slo + 0.75 * to.rtol, mid);
                if (shi - sc < close) sc = std::max(shi - 0.75 * to.rtol, mid);
            }
        }
        prev_newton = use_newton;
        if (!use_newton) prev_step = INFINITY;
        const double tc = std::exp(sc);
        if (!(tc > lo.t && tc < hi.t)) break;
        CHK(tplus_eval(c, X, n, m, tc, o, newton, w_cur, cur, solves));
        if (use_newton) ++newton_steps;
        last = cur;
        if (cur.minw < 0.0) {
            lo = cur;
        } else {
            accept_hi(cur);
            if (cur.minw < eps) break;  // halting rule: 0 <= min w < eps
        }
    }
    *t_plus = hi.t;
    if (w_out) {
        launch_copy(c->stream, w_hi, w_out, n);
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    if (info) {
        info->t_plus = hi.t;
        info->t_bound = tb;
        info->d_min = dmin;
        info->min_w = hi.minw;
        info->t_bracket_lo = lo.t;
        info->t_bracket_hi = hi.t;
        info->solves = solves;
        info->newton_steps = newton_steps;
        info->no_sign_change = 0;
        info->status = MAG_OK;
    }
    return MAG_OK;
}

int mag_dwdt(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, double *w, double *dwdt,
             const mag_opts *opts)
{
    if (!c || !dwdt || !valid_args(X, n, m, t)) return MAG_EINVAL;
    if (m > pair_max_dim()) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    mag_opts o;
    if (opts) o = *opts;
    else mag_opts_default(&o);
    const int restart = std::max(1, o.gmres_restart);
    CHK(ensure_solver(c, n, m, restart));
    CHK(check_points(c, X, n, m));
    const int64_t npad = round_up(n, kPad);
    CHK(ensure_ctx_factor(c, n));
    CHK(ensure_aux(c, npad));
    Factor32 F = ctx_factor(c, n);
    CHK(factor_fp32(c, X, n, m, t, F, nullptr, nullptr));
    double *wv = (double *)c->aux.p + npad;
    double *d = (double *)c->aux.p + 2 * npad;
    RefineStats st;
    int rc = refine_solve(c, X, n, m, t, F, nullptr, 1.0, wv, o, st);
    if (rc != MAG_OK) return rc;
    rc = dwdt_with_factor(c, X, n, m, t, F, wv, d, o, st);
    if (rc != MAG_OK) return rc;
    if (w) HIPCHK(hipMemcpyAsync(w, wv, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dwdt, d, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return MAG_OK;
}

// ---- weighting at scale zero (Appendix C.1, eq. scaleZero) ---------------------

int mag_weighting_zero(mag_ctx *c, const double *X, int64_t n, int32_t m, double *w, const mag_opts *opts,
                       mag_info *info, double *sum_dinv, double *c_used)
{
    if (info) std::memset(info, 0, sizeof(*info));
    if (!c || !X || !w || n < 1 || m < 1 || m > 16) return MAG_EINVAL;
    mag_opts o;
    if (opts) o = *opts;
    else mag_opts_default(&o);
    if (o.solver != MAG_AUTO && o.solver != MAG_FP32_IR) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    const int restart = std::max(1, o.gmres_restart);
    CHK(ensure_solver(c, n, m, restart));
    CHK(check_points(c, X, n, m, false));
    hipStream_t s = c->stream;
    if (n == 1) {
        launch_fill(s, w, 1, 1.0);
        HIPCHK(hipStreamSynchronize(s));
        if (info) {
            info->magnitude = 1.0;
            info->min_w = 1.0;
        }
        if (sum_dinv) *sum_dinv = INFINITY;
        if (c_used) *c_used = 0.0;
        return MAG_OK;
    }
    if (o.solver == MAG_AUTO && !auto_dense(c, n)) return MAG_ENOMEM;
    // c: twice the largest distance from the centroid, an upper bound of the diameter
    std::vector<double> hx((size_t)n * m);
    HIPCHK(hipMemcpyAsync(hx.data(), X, sizeof(double) * hx.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<double> cen(m, 0.0);
    for (int64_t j = 0; j < n; ++j)
        for (int l = 0; l < m; ++l) cen[l] += hx[(size_t)j * m + l];
    for (int l = 0; l < m; ++l) cen[l] /= (double)n;
    double rad2 = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double q = 0.0;
        for (int l = 0; l < m; ++l) {
            const double e = hx[(size_t)j * m + l] - cen[l];
            q += e * e;
        }
        rad2 = std::max(rad2, q);
    }
    double cs = 2.0 * std::sqrt(rad2);
    if (!(cs > 0.0) || !std::isfinite(cs)) return MAG_ENOTPD;  // every point coincides
    CHK(ensure_ctx_factor(c, n));
    Factor32 F = ctx_factor(c, n);
    for (int attempt = 0; attempt < 2; ++attempt) {
        CHK(factor_fp32(c, X, n, m, cs, F, nullptr, nullptr, kKernShiftDist));
        if (!F.shifted || attempt == 1) break;
        cs *= 2.0;  // c may be below 1 / (1^T d^{-1} 1): B indefinite
    }
    Vecs v;
    CHK(carve_vecs(c, F.npad, restart, v));
    RefineStats st;
    const int rc = refine_solve(c, X, n, m, cs, F, nullptr, 1.0, v.best, o, st, kKernShiftDist);
    if (rc != MAG_OK && rc != MAG_ENOCONV) return rc;
    double beta, mn;
    int64_t am;
    CHK(summarize(c, v.best, n, beta, mn, am));
    if (!(beta != 0.0) || !std::isfinite(beta)) return MAG_EINTERNAL;
    launch_scale(s, v.best, 1.0 / beta, w, n, n);
    double sw;
    CHK(summarize(c, w, n, sw, mn, am));
    if (info) {
        info->outer_iters = st.outer;
        info->gmres_iters = st.inner;
        info->shifted = F.shifted;
        info->shift = F.shift;
        info->resid_inf = st.resid;
        info->magnitude = sw;
        info->min_w = mn;
        info->argmin_w = am;
    }
    if (sum_dinv) *sum_dinv = beta / (cs * beta - 1.0);
    if (c_used) *c_used = cs;
    return rc;
}

// ---- extreme eigenvalues (Section 4.2 positive-definiteness check) -----------

void mag_eig_opts_default(mag_eig_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_iter = 80;
    o->rtol = 1e-8;
}

int mag_eig_extremes(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, const double *v0,
                     const mag_eig_opts *eopts, const mag_opts *opts, mag_eig_info *info)
{
    if (!c || !info || !valid_args(X, n, m, t)) return MAG_EINVAL;
    mag_eig_opts eo;
    if (eopts) eo = *eopts;
    else mag_eig_opts_default(&eo);
    const int max_iter = eo.max_iter > 0 ? eo.max_iter : 80;
    const double rtol = eo.rtol > 0 ? eo.rtol : 1e-8;
    if (max_iter > 256) return MAG_EINVAL;
    mag_opts o;
    if (opts) o = *opts;
    else mag_opts_default(&o);
    if (o.solver != MAG_AUTO && o.solver != MAG_FP32_IR) return MAG_EINVAL;
    std::memset(info, 0, sizeof(*info));
    HIPCHK(hipSetDevice(c->device));
    const int restart = std::max(1, o.gmres_restart);
    CHK(ensure_solver(c, n, m, restart));
    // the orthogonalisation's dot products against up to max_iter + 1 vectors
    CHK(ensure(c, c->partial, sizeof(double) * (blas1_partial_doubles(max_iter + 2) + 64)));
    CHK(check_points(c, X, n, m, false));
    if (o.solver == MAG_AUTO && !auto_dense(c, n)) return MAG_ENOMEM;
    const int64_t npad = round_up(n, kPad);
    CHK(ensure_ctx_factor(c, n));
    // basis (max_iter + 1 vectors), the work vector, start vector and device scalars
    CHK(ensure(c, c->eig, sizeof(double) * ((size_t)(max_iter + 3) * npad + 2 * (max_iter + 2) + 64)));
    hipStream_t s = c->stream;
    double *Q = (double *)c->eig.p;
    double *u = Q + (size_t)(max_iter + 1) * npad;
    double *q0 = u + npad;
    double *dev = q0 + npad;
    double *partial = (double *)c->partial.p;
    if (v0) {
        launch_scale(s, v0, 1.0, q0, n, npad);
    } else {
        launch_golden(s, q0, n, npad);
    }
    launch_nrm2(s, q0, npad, partial, dev);
    HIPCHK(hipMemcpyAsync(c->host_scalars, dev, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!(c->host_scalars[0] > 0.0) || !std::isfinite(c->host_scalars[0])) return MAG_EINVAL;
    const double q0norm = c->host_scalars[0];

    // lambda_max: Lanczos on Z (matrix-free FP64 products)
    LanczosResult top;
    const auto zop = [&](const double *in, double *out) -> int {
        launch_zmv(s, X, n, m, t, in, out, nullptr, 0, partial, nullptr);
        return MAG_OK;
    };
    launch_scale(s, q0, 1.0 / q0norm, Q, npad, npad);
    CHK(lanczos_top(c, npad, zop, Q, u, dev, max_iter, rtol, top));

    // lambda_min: Lanczos on Z^{-1} through the FP32 factor + refinement
    Factor32 F = ctx_factor(c, n);
    CHK(factor_fp32(c, X, n, m, t, F, nullptr, nullptr));
    int solve_steps = 0, solve_rc = MAG_OK;
    const auto iop = [&](const double *in, double *out) -> int {
        RefineStats st;
        const int rc = refine_solve(c, X, n, m, t, F, in, 1.0, out, o, st);
        solve_steps += st.outer;
        if (rc == MAG_ENOCONV) {
            solve_rc = rc;
            return MAG_OK;
        }
        return rc;
    };
    LanczosResult bot;
    launch_scale(s, q0, 1.0 / q0norm, Q, npad, npad);
    CHK(lanczos_top(c, npad, iop, Q, u, dev, max_iter, rtol, bot));

    info->lambda_max = top.theta;
    info->resid_max = top.resid;
    info->iters_max = top.iters;
    info->lambda_min = (bot.theta > 0.0) ? 1.0 / bot.theta : 0.0;
    info->resid_min = bot.resid;
    info->iters_min = bot.iters;
    info->cond = (bot.theta > 0.0) ? top.theta * bot.theta : INFINITY;
    info->converged = (top.converged ? 1 : 0) | (bot.converged ? 2 : 0);
    info->solve_steps = solve_steps;
    return solve_rc;
}

// ---- adjoint ----------------------------------------------------------------

int mag_weighting_fwd(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, double *w,
                      mag_factor **keep, const mag_opts *opts, mag_info *info)
{
    if (info) std::memset(info, 0, sizeof(*info));
    if (!c || !w || !keep || !valid_args(X, n, m, t)) return MAG_EINVAL;
    *keep = nullptr;
    HIPCHK(hipSetDevice(c->device));
    mag_opts o;
    if (opts) o = *opts;
    else mag_opts_default(&o);
    CHK(ensure_solver(c, n, m, std::max(1, o.gmres_restart)));
    CHK(check_points(c, X, n, m));
    {
        const size_t np = (size_t)round_up(n, kPad);
        CHK(ctx_may_allocate(c, sizeof(float) * (np * np + np * kTile + near_q_floats(np))));
    }
    mag_factor *f = new mag_factor();
    f->device = c->device;
    f->n = n;
    f->m = m;
    f->t = t;
    f->F.npad = round_up(n, kPad);
    if (hipMalloc((void **)&f->F.A, sizeof(float) * (size_t)f->F.npad * f->F.npad) != hipSuccess ||
        hipMalloc((void **)&f->F.dinv,
                  sizeof(float) * ((size_t)f->F.npad * kTile + near_q_floats(f->F.npad))) != hipSuccess) {
        (void)hipGetLastError();
        mag_factor_free(f);
        return MAG_ENOMEM;
    }
    f->F.nq = f->F.dinv + (size_t)f->F.npad * kTile;
    int rc;
    if (n == 1) {
        launch_fill(c->stream, w, 1, 1.0);
        HIPCHK(hipStreamSynchronize(c->stream));
        // factor of [1] padded with identity: build it through the normal path
        rc = factor_fp32(c, X, n, m, t, f->F, nullptr, nullptr);
        if (info) {
            info->magnitude = 1.0;
            info->min_w = 1.0;
        }
    } else {
        rc = solve_fp32_ir(c, X, n, m, t, w, o, info, &f->F);
    }
    if (info) info->status = rc;
    if (rc != MAG_OK) {
        mag_factor_free(f);
        return rc;
    }
    *keep = f;
    return MAG_OK;
}

int mag_weighting_vjp(mag_ctx *c, mag_factor *f, const double *X, int64_t n, int32_t m, double t,
                      const double *w, double gM, const double *gw, double *dX, double *dt,
                      const mag_opts *opts)
{
    if (!c || !f || !w || !valid_args(X, n, m, t)) return MAG_EINVAL;
    if (f->n != n || f->m != m || f->t != t || f->device != c->device) return MAG_EINVAL;
    if (m > pair_max_dim()) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    mag_opts o;
    if (opts) o = *opts;
    else mag_opts_default(&o);
    hipStream_t s = c->stream;
    const int64_t npad = f->F.npad;
    CHK(ensure_solver(c, n, m, std::max(1, o.gmres_restart)));
    CHK(ensure_aux(c, npad));
    double *aux = (double *)c->aux.p;
    double *u = aux;              // (D o Z) w
    double *lam = aux + npad;     // lambda
    double *wv = aux + 2 * npad;  // w padded
    double *rhs = aux + 3 * npad;
    double *partial = (double *)c->partial.p;
    launch_scale(s, w, 1.0, wv, n, npad);
    if (gw) {
        // lambda = Z^{-1} (gM 1 + gw), with the kept factor
        launch_affine_ones(s, gw, gM, rhs, n, npad);
        double *amax = (double *)c->partial.p + blas1_partial_doubles(3) + 8;
        launch_amax(s, rhs, npad, partial, amax);
        HIPCHK(hipMemcpyAsync(c->host_scalars + 42, amax, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        RefineStats st;
        int rc = refine_solve(c, X, n, m, t, f->F, rhs, c->host_scalars[42], lam, o, st);
        if (rc != MAG_OK) return rc;
    } else {
        launch_scale(s, wv, gM, lam, n, npad);  // lambda = gM w
    }
    if (dt) {
        launch_dzmv(s, X, n, m, t, wv, u, partial);
        double *h = (double *)c->partial.p + blas1_partial_doubles(3) + 16;
        launch_multidot(s, u, npad, 1, lam, npad, partial, h);
        HIPCHK(hipMemcpyAsync(c->host_scalars + 43, h, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (dX) launch_gradx(s, X, n, m, t, wv, lam, dX, partial);
    HIPCHK(hipStreamSynchronize(s));
    if (dt) *dt = c->host_scalars[43];
    return MAG_OK;
}

void mag_factor_free(mag_factor *f)
{
    if (!f) return;
    hipSetDevice(f->device);
    if (f->F.A) hipFree(f->F.A);
    if (f->F.dinv) hipFree(f->F.dinv);
    delete f;
}

int mag_dzmatvec(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, const double *v,
                 double *y)
{
    if (!c || !v || !y || !valid_args(X, n, m, t)) return MAG_EINVAL;
    if (m > pair_max_dim()) return MAG_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    CHK(ensure_solver(c, n, m, 1));
    const int64_t npad = round_up(n, kPad);
    CHK(ensure_aux(c, npad));
    double *aux = (double *)c->aux.p;
    launch_scale(c->stream, v, 1.0, aux + npad, n, npad);
    launch_dzmv(c->stream, X, n, m, t, aux + npad, aux, (double *)c->partial.p);
    HIPCHK(hipMemcpyAsync(y, aux, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return MAG_OK;
}

}  // extern "C"
