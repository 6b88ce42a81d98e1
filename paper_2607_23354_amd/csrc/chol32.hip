// chol32.hip -- blocked right-looking FP32 Cholesky of Z on MFMA.
//
// Z is symmetric positive definite for distinct Euclidean points (Sections 2
// and 3.2), so Z = L L^T exists; this factor is computed in FP32 and used as
// the preconditioner of the FP64 refinement.  For each panel of nb = 512
// columns (or 256, the tunable choice) starting at k (256 for a last,
// narrower panel), made of 128-column sub-panels s:
//   1. potrf128   factor of the 128 x 128 diagonal block and its inverse
//   2. trsm       rows below:  L21 = A21 * inv(L11)^T     (MFMA, in place),
//                 with L21^T written into the upper triangle
//   3. update     the panel's later sub-panels by this one (K = 128)
// and, panels taken in pairs, 4. the trailing update A22 -= L21 L21^T of both
// panels at once (K = 2 nb, lower tiles only), after a strip update of the
// second panel's columns by the first.  A deep K in step 4 amortises the load
// and store of each C tile over more MFMA work; steps 2, 3 and the strip run
// on 64-row tiles (twice the workgroups of 128-row ones, which keeps more CUs
// busy in the late panels, where a 128-row tiling leaves most of them idle).
// The inverses of the diagonal 128-blocks are kept (dinv) for the
// preconditioner's triangular solves.
#include "internal.hpp"

#include <algorithm>
#include <vector>

namespace mag {


namespace {

// Steps 1-3 for the panel of nb columns at k (its trailing rows already updated
// by every earlier panel).
void factor_panel(hipStream_t s, float *A, int64_t npad, int64_t k, int64_t nb, float *dinv, int *status)
{
    const int64_t T = kTile;
    const int64_t nsub = nb / T;
    for (int64_t sub = 0; sub < nsub; ++sub) {
        const int64_t kk = k + sub * T;
        float *Linv = dinv + (kk / T) * T * T;
        launch_potrf128(s, A, npad, kk, Linv, status);
        const int64_t below = npad - kk - T;
        if (below > 0) {
            float *A21 = A + kk * npad + kk + T;
            float *A12 = A + (kk + T) * npad + kk;  // upper triangle: L21^T
            launch_gemm_rows64(s, A21, npad, A21, npad, Linv, T, below, T, T, kGemmSetT, A12);
        }
        if (sub + 1 < nsub) {
            // the panel's remaining sub-panels (rows kk+T ..) by this sub-panel;
            // tiles above their diagonal are rewritten later by their own trsm
            float *C = A + (kk + T) * npad + kk + T;
            const float *P = A + kk * npad + kk + T;
            launch_gemm_rows64(s, C, npad, P, npad, P, npad, below, (nsub - sub - 1) * T, T, kGemmSub);
        }
    }
}

}  // namespace

// Factor the padded npad x npad FP32 matrix A (column-major, ld = npad) in place.
// timer (optional) records an event pair around every trailing update.
//
// Panels go in pairs (p, p+1): after panel p, only panel p+1's columns are
// updated by it (a strip, M x nb x nb); panel p+1 is factored; then one trailing
// update with K = 2 nb applies both panels to the rest.  Each tile of the large
// trailing block is read and written once per two panels.
void chol32_factor(hipStream_t s, float *A, int64_t npad, int64_t n, float *dinv, int *status,
                   FactorTimer *timer, int nb_max)
{
    const int64_t kNb = (nb_max == 256) ? 256 : 512;
    int64_t k = 0;
    while (k < npad) {
        const int64_t nb = std::min<int64_t>(kNb, npad - k);
        factor_panel(s, A, npad, k, nb, dinv, status);
        const int64_t k2 = k + nb;
        if (k2 >= npad) break;
        const int64_t nb2 = std::min<int64_t>(kNb, npad - k2);
        {
            // strip: panel p+1's columns (all rows from k2) by panel p; the tiles above
            // the 128-diagonal of its diagonal block are rewritten by its own trsm
            float *C = A + k2 * npad + k2;
            const float *P = A + k * npad + k2;
            launch_gemm_rows64(s, C, npad, P, npad, P, npad, npad - k2, nb2, nb, kGemmSub);
        }
        factor_panel(s, A, npad, k2, nb2, dinv, status);
        const int64_t k3 = k2 + nb2;
        const int64_t trail = npad - k3;
        if (trail > 0) {
            const int64_t K = nb + nb2;  // both panels, contiguous columns k .. k3-1
            float *C = A + k3 * npad + k3;
            const float *P = A + k * npad + k3;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timer) {
                if (timer->used + 2 > timer->ev.size()) {
                    for (int q = 0; q < 64; ++q) {
                        hipEvent_t e;
                        hipEventCreate(&e);
                        timer->ev.push_back(e);
                    }
                }
                e0 = timer->ev[timer->used++];
                e1 = timer->ev[timer->used++];
                // algorithmic flops of the trailing update restricted to the true n
                const int64_t nt = n - k3;
                timer->flops.push_back(nt > 0 ? (double)K * (double)nt * (double)(nt + 1) : 0.0);
                hipEventRecord(e0, s);
            }
            launch_syrk_lower(s, C, npad, P, npad, trail, K);
            if (timer) hipEventRecord(e1, s);
        }
        k = k3;
    }
}

int size_bucket(int64_t npad)
{
    int b = 0;
    while (b < 63 && ((int64_t)1 << b) < npad) ++b;
    return b;
}

int panel_width(const mag_ctx *ctx, int64_t npad)
{
    const int v = ctx ? ctx->tune_panel[size_bucket(npad)] : 0;
    return (v == 256 || v == 512) ? v : 512;
}

}  // namespace mag
