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
#include <cmath>
#include <cstring>
#include <vector>

namespace mag {


int ensure(mag_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes <= b.bytes) return MAG_OK;
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

// Validate the coordinates: finite, and no duplicate points (Z would be
// singular).  One host sync.
int check_points(mag_ctx *ctx, const double *X, int64_t n, int m)
{
    int *status = (int *)ctx->ints.p;
    CHK(ensure(ctx, ctx->partial, sizeof(double) * std::max<size_t>(dmin_partial_doubles(n) + 8, 64)));
    double *partial = (double *)ctx->partial.p;
    launch_fill_ints(ctx->stream, status, 8, 0);
    launch_check_finite(ctx->stream, X, n * (int64_t)m, status);
    double *dmin2 = partial + dmin_partial_doubles(n);
    if (n >= 2) launch_dmin2(ctx->stream, X, n, m, partial, nullptr, dmin2);
    HIPCHK(hipMemcpyAsync(ctx->host_scalars, status, 8 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    if (n >= 2)
        HIPCHK(hipMemcpyAsync(ctx->host_scalars + 8, dmin2, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const int *hs = (const int *)ctx->host_scalars;
    if (hs[kStNonFinite]) return MAG_EINVAL;
    if (n >= 2 && !(ctx->host_scalars[8] > 0.0)) return MAG_ENOTPD;
    return MAG_OK;
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

// FP32-factor + FP64 GMRES iterative refinement.  Returns status; w holds the
// best iterate.
int solve_fp32_ir(mag_ctx *ctx, const double *X, int64_t n, int m, double t, double *w,
                  const mag_opts &o, mag_info *info)
{
    hipStream_t s = ctx->stream;
    const int64_t npad = round_up(n, kPad);
    const int restart = std::max(1, o.gmres_restart);
    CHK(ensure_common(ctx, n, restart));
    CHK(ensure(ctx, ctx->factor, sizeof(float) * (size_t)npad * (size_t)npad));
    CHK(ensure(ctx, ctx->dinv, sizeof(float) * (size_t)npad * kTile));
    // vectors: V (restart+1), wv, r, z, ytmp, u, best, dev scalars
    const int nvec = restart + 1 + 6;
    CHK(ensure(ctx, ctx->vecs, sizeof(double) * ((size_t)nvec * npad + 256)));
    float *A = (float *)ctx->factor.p;
    float *dinv = (float *)ctx->dinv.p;
    double *V = (double *)ctx->vecs.p;
    double *wv = V + (size_t)(restart + 1) * npad;
    double *r = wv + npad;
    double *z = r + npad;
    double *ytmp = z + npad;
    double *u = ytmp + npad;
    double *best = u + npad;
    double *dsc = best + npad;  // device scalars: [0] norm, [1..] h, ...
    double *hdev = dsc + 8;     // up to 2*(restart+1) + 2
    double *partial = (double *)ctx->partial.p;
    int *ints = (int *)ctx->ints.p;
    int *status = ints + kIntStatus;
    int *counters = ints + kIntCounters;
    double *hs = ctx->host_scalars;

    Timer tm;
    tm.start(o.profile != 0, s);
    FactorTimer ft;
    tm.mark(0);

    // ---- factor (with diagonal-shift retries on FP32 breakdown) ----
    double shift = 0.0;
    int shifted = 0;
    for (int attempt = 0;; ++attempt) {
        launch_fill_ints(s, status, 8, 0);
        launch_tilegen32(s, X, n, m, t, A, npad, (float)shift);
        if (attempt == 0) tm.mark(1);
        ft.used = 0;
        ft.flops.clear();
        chol32_factor(s, A, npad, n, dinv, status, o.profile ? &ft : nullptr);
        HIPCHK(hipMemcpyAsync(hs, status, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (((const int *)hs)[kStBreakdown] == 0) break;
        if (attempt >= 6) return MAG_ENOTPD;
        shift = (shift == 0.0) ? 1e-6 * std::max<double>(1.0, std::sqrt((double)n)) : shift * 10.0;
        shifted = 1;
    }
    tm.mark(2);

    // ---- refinement ----
    const double tol = o.tol > 0 ? o.tol : 1e-12;
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-10;
    int outer = 0, inner_total = 0;
    double rnorm = INFINITY, best_norm = INFINITY;
    int rc = MAG_ENOCONV;

    // w0 = M^{-1} 1
    launch_fill(s, r, npad, 0.0);
    launch_fill(s, r, n, 1.0);
    launch_prec_apply(s, A, npad, dinv, r, ytmp, wv, counters, status);

    Gmres G;
    G.restart = restart;
    G.H.assign((size_t)(restart + 1) * restart, 0.0);
    G.cs.assign(restart, 0.0);
    G.sn.assign(restart, 0.0);
    G.g.assign(restart + 1, 0.0);
    std::vector<double> hbuf(2 * (restart + 2) + 2);

    for (outer = 0; outer < std::max(1, o.max_outer); ++outer) {
        launch_zmv(s, X, n, m, t, wv, r, nullptr, 1, partial, dsc);
        HIPCHK(hipMemcpyAsync(hs, dsc, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hs + 8, status, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (((const int *)(hs + 8))[kStSpinTimeout]) return MAG_EINTERNAL;
        const double prev = rnorm;
        rnorm = hs[0];
        if (!(rnorm < best_norm)) {
            // no progress: stop with the best iterate
            break;
        }
        best_norm = rnorm;
        launch_copy(s, wv, best, npad);
        if (rnorm <= tol) {
            rc = MAG_OK;
            break;
        }
        if (outer > 0 && rnorm > 0.5 * prev) break;  // stagnation
        if (inner_total >= o.max_gmres) break;
        // GMRES(restart) on M^{-1} Z d = M^{-1} r, d0 = 0
        double *V0 = V;
        launch_prec_apply(s, A, npad, dinv, r, ytmp, z, counters, status);
        launch_nrm2(s, z, npad, partial, dsc + 1);
        HIPCHK(hipMemcpyAsync(hs + 1, dsc + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double beta = hs[1];
        if (!(beta > 0.0) || !std::isfinite(beta)) break;
        launch_scale_inv(s, z, V0, npad, dsc + 1);
        std::fill(G.H.begin(), G.H.end(), 0.0);
        std::fill(G.g.begin(), G.g.end(), 0.0);
        G.g[0] = beta;
        int kdone = 0;
        for (int k = 0; k < restart && inner_total < o.max_gmres; ++k) {
            double *Vk = V + (size_t)k * npad;
            double *Vk1 = V + (size_t)(k + 1) * npad;
            launch_zmv(s, X, n, m, t, Vk, u, nullptr, 0, partial, nullptr);
            launch_prec_apply(s, A, npad, dinv, u, ytmp, Vk1, counters, status);
            // classical Gram-Schmidt, twice
            launch_multidot(s, V, npad, k + 1, Vk1, npad, partial, hdev);
            launch_multi_axpy(s, V, npad, k + 1, hdev, Vk1, npad, -1.0);
            launch_multidot(s, V, npad, k + 1, Vk1, npad, partial, hdev + (k + 1));
            launch_multi_axpy(s, V, npad, k + 1, hdev + (k + 1), Vk1, npad, -1.0);
            launch_nrm2(s, Vk1, npad, partial, hdev + 2 * (k + 1));
            HIPCHK(hipMemcpyAsync(hbuf.data(), hdev, sizeof(double) * (2 * (k + 1) + 1),
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            const double hk1 = hbuf[2 * (k + 1)];
            double *Hk = G.H.data() + (size_t)k * (restart + 1);
            for (int i = 0; i <= k; ++i) Hk[i] = hbuf[i] + hbuf[k + 1 + i];
            Hk[k + 1] = hk1;
            if (hk1 > 0.0) launch_scale_inv(s, Vk1, Vk1, npad, hdev + 2 * (k + 1));
            // apply previous rotations, then a new one
            for (int i = 0; i < k; ++i) {
                const double a = Hk[i], b = Hk[i + 1];
                Hk[i] = G.cs[i] * a + G.sn[i] * b;
                Hk[i + 1] = -G.sn[i] * a + G.cs[i] * b;
            }
            const double a = Hk[k], b = Hk[k + 1];
            const double rr = std::hypot(a, b);
            G.cs[k] = (rr > 0) ? a / rr : 1.0;
            G.sn[k] = (rr > 0) ? b / rr : 0.0;
            Hk[k] = rr;
            Hk[k + 1] = 0.0;
            G.g[k + 1] = -G.sn[k] * G.g[k];
            G.g[k] = G.cs[k] * G.g[k];
            ++inner_total;
            kdone = k + 1;
            if (std::fabs(G.g[k + 1]) <= inner_tol * beta || !(hk1 > 0.0)) break;
        }
        // y = H^{-1} g (upper triangular kdone x kdone)
        std::vector<double> y(kdone, 0.0);
        for (int i = kdone - 1; i >= 0; --i) {
            double acc = G.g[i];
            for (int j = i + 1; j < kdone; ++j) acc -= G.H[(size_t)j * (restart + 1) + i] * y[j];
            y[i] = acc / G.H[(size_t)i * (restart + 1) + i];
        }
        HIPCHK(hipMemcpyAsync(hdev, y.data(), sizeof(double) * kdone, hipMemcpyHostToDevice, s));
        launch_multi_axpy(s, V, npad, kdone, hdev, wv, npad, 1.0);
    }
    tm.mark(3);
    // return the best iterate
    launch_copy(s, best, w, n);
    launch_sum_min(s, best, n, partial, dsc + 2);
    HIPCHK(hipMemcpyAsync(hs + 2, dsc + 2, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    tm.mark(4);
    if (info) {
        info->outer_iters = outer + (rc == MAG_OK ? 1 : 0);
        info->gmres_iters = inner_total;
        info->shifted = shifted;
        info->shift = shift;
        info->resid_inf = best_norm;
        info->magnitude = hs[2];
        info->min_w = hs[3];
        info->argmin_w = (int64_t)hs[4];
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
    o->leaf = 256;
    o->max_rank = 64;
    o->oversample = 16;
    o->profile = 0;
    o->seed = 0x9E3779B97F4A7C15ull;
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
    if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
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
    for (DevBuf *b : {&c->factor, &c->dinv, &c->vecs, &c->partial, &c->ints})
        if (b->p) hipFree(b->p);
    if (c->blas) rocblas_destroy_handle((rocblas_handle)c->blas);
    if (c->host_scalars) hipHostFree(c->host_scalars);
    if (c->own_stream) hipStreamDestroy(c->own_stream);
    delete c;
}

int mag_set_stream(mag_ctx *c, void *stream)
{
    if (!c) return MAG_EINVAL;
    c->stream = stream ? (hipStream_t)stream : c->own_stream;
    return MAG_OK;
}

int64_t mag_padded_size(int64_t n) { return n < 1 ? 0 : round_up(n, kPad); }

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
    int rc = check_points(c, X, n, m);
    if (rc == MAG_OK && n == 1) {
        launch_fill(c->stream, w, 1, 1.0);
        HIPCHK(hipStreamSynchronize(c->stream));
        if (info) {
            info->magnitude = 1.0;
            info->min_w = 1.0;
        }
    } else if (rc == MAG_OK) {
        switch (o.solver) {
        case MAG_FP64_DENSE: rc = solve_fp64_dense(c, X, n, m, t, w, o, info); break;
        case MAG_AUTO:
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
    chol32_factor(c->stream, L, npad, n, dinv, status, nullptr);
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
    CHK(ensure(c, c->vecs, sizeof(double) * ((size_t)npad * 3 + 256)));
    double *rb = (double *)c->vecs.p;
    double *yt = rb + npad;
    double *zb = yt + npad;
    int *ints = (int *)c->ints.p;
    launch_fill_ints(c->stream, ints, 8, 0);
    launch_fill(c->stream, rb, npad, 0.0);
    HIPCHK(hipMemcpyAsync(rb, r, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    launch_prec_apply(c->stream, L, npad, dinv, rb, yt, zb, ints + kIntCounters, ints);
    HIPCHK(hipMemcpyAsync(z, zb, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->host_scalars, ints, 8 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (((const int *)c->host_scalars)[kStSpinTimeout]) return MAG_EINTERNAL;
    return MAG_OK;
}

}  // extern "C"
