// chol64.hip -- blocked right-looking FP64 Cholesky of Z on the FP64 matrix
// cores: the dense comparator of the FP32 factor + FP64 refinement.
//
// Z is symmetric positive definite for distinct Euclidean points (Sections 2
// and 3.2).  The schedule is that of the FP32 factor, with 64-column
// sub-panels (an FP64 diagonal block and its inverse fit one workgroup's LDS at
// that size) and 256-column panels taken in pairs.  For the panel of nb = 256
// columns at k, made of 64-column sub-panels:
//   1. potrf64   factor of the 64 x 64 diagonal block and its inverse
//   2. trsm      rows below:  L21 = A21 * inv(L11)^T     (MFMA, in place),
//                with L21^T written into the upper triangle
//   3. update    the panel's later sub-panels by this one (K = 64)
// and, per pair of panels, 4. a strip update of the second panel's columns by
// the first (K = 256, 64-tiles: four tile columns fill the device where two
// 128-tile columns would occupy half of it), then one trailing update
// A22 -= L21 L21^T of both panels at once (K = 512, lower 128-tiles only).  The inverses of the
// diagonal 64-blocks are kept (dinv) for the triangular solves.
#include "internal.hpp"

#include <algorithm>

namespace mag {
namespace {

constexpr int64_t kSub = 64;    // sub-panel width = diagonal block
constexpr int64_t kNb64 = 256;  // panel width

void factor_panel64(hipStream_t s, double *A, int64_t npad, int64_t k, int64_t nb, double *dinv, int *status)
{
    const int64_t nsub = nb / kSub;
    for (int64_t sub = 0; sub < nsub; ++sub) {
        const int64_t kk = k + sub * kSub;
        double *Linv = dinv + (kk / kSub) * kSub * kSub;
        launch_potrf64(s, A, npad, kk, Linv, status);
        const int64_t below = npad - kk - kSub;
        if (below > 0) {
            double *A21 = A + kk * npad + kk + kSub;
            double *A12 = A + (kk + kSub) * npad + kk;  // upper triangle: L21^T
            launch_gemm64(s, 64, A21, npad, A21, npad, Linv, kSub, below, kSub, kSub, kGemmSetT, A12);
        }
        if (sub + 1 < nsub) {
            // the panel's remaining sub-panels (rows kk+64 ..) by this sub-panel;
            // tiles above their diagonal are rewritten later by their own trsm
            double *C = A + (kk + kSub) * npad + kk + kSub;
            const double *P = A + kk * npad + kk + kSub;
            launch_gemm64(s, 64, C, npad, P, npad, P, npad, below, (nsub - sub - 1) * kSub, kSub, kGemmSub, nullptr);
        }
    }
}

}  // namespace

void chol64_factor(hipStream_t s, double *A, int64_t npad, int64_t n, double *dinv, int *status, FactorTimer *timer)
{
    int64_t k = 0;
    while (k < npad) {
        const int64_t nb = std::min<int64_t>(kNb64, npad - k);
        factor_panel64(s, A, npad, k, nb, dinv, status);
        const int64_t k2 = k + nb;
        if (k2 >= npad) break;
        const int64_t nb2 = std::min<int64_t>(kNb64, npad - k2);
        {
            // strip: panel p+1's columns (all rows from k2) by panel p; the tiles above
            // the diagonal blocks are rewritten by the second panel's own trsm
            double *C = A + k2 * npad + k2;
            const double *P = A + k * npad + k2;
            launch_gemm64(s, 64, C, npad, P, npad, P, npad, npad - k2, nb2, nb, kGemmSub, nullptr);
        }
        factor_panel64(s, A, npad, k2, nb2, dinv, status);
        const int64_t k3 = k2 + nb2;
        const int64_t trail = npad - k3;
        if (trail > 0) {
            const int64_t K = nb + nb2;  // both panels, contiguous columns k .. k3-1
            double *C = A + k3 * npad + k3;
            const double *P = A + k * npad + k3;
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
            launch_syrk64_lower(s, C, npad, P, npad, trail, K);
            if (timer) hipEventRecord(e1, s);
        }
        k = k3;
    }
}

}  // namespace mag
