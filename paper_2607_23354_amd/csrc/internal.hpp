// internal.hpp -- shared declarations of libmag's HIP translation units.
//
// Storage conventions used by every kernel:
//   * X        caller's points, row-major n x m FP64 (device).
//   * factor   FP32, column-major, leading dimension npad = n rounded up to
//              a multiple of 256.  Element (i, j) at A[j * npad + i].  The
//              factor L is built in the lower triangle; as each panel is
//              finished its transpose is written into the upper triangle, so
//              the backward substitution streams L^T with the same access
//              pattern as the forward one.  Rows/columns >= n are an identity
//              padding, so every kernel works on whole tiles.
//   * vectors  FP64, length npad, zero in the padding.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "mag.h"

namespace mag {

constexpr int kPad = 256;      // npad multiple (panel width of the factor)
constexpr int kTile = 128;     // MFMA tile edge and diagonal-block size
constexpr int kPanel = 256;    // npad multiple; panel width of the batched factorisation

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// ---- device buffer that grows on demand ------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// The kernel matrix a factor or product is built from: Z = exp[-t d] (Section
// 2), or c 1 1^T - d for the weighting at scale zero (eq. scaleZero), with c in
// the place of t.
constexpr int kKernExp = 0, kKernShiftDist = 1;

// Status words written by kernels (device memory, zeroed per call).
enum StatusWord : int {
    kStBreakdown = 0,    // FP32 Cholesky met a non-positive pivot (index+1)
    kStSpinTimeout = 1,  // a bounded spin-wait gave up (should never happen)
    kStNonFinite = 2,    // non-finite coordinate seen
    kStDuplicate = 3,    // two points at distance 0 seen by the FP32 tile generator
    kStCount = 8
};

// ---- batched problems --------------------------------------------------------
// One descriptor per problem of a batch (device array).  A batched launch takes
// a work list: items i = 0..na-1, problem plist[i], work units
// [pref[i], pref[i+1]) of the flat block index; bfind() maps a block to its item.
struct BProb {
    const double *X;
    int64_t n, npad;
    double t;
    double shift;     // diagonal shift of the FP32 factor (0 unless it broke down)
    float *A;         // FP32 factor, npad x npad column-major
    float *dinv;      // inverses of the 128-diagonal blocks
    double *vec;      // this problem's FP64 vectors: slot j at vec + j * npad
    double *scal;     // this problem's device scalars
    double *partial;  // this problem's split-reduction buffer
    int *ints;        // status [0, 64) and preconditioner counters [64, ...)
    int32_t m;
    int32_t active;   // 0: skip (finished)
};

struct BWork {
    const int *plist;
    const int64_t *pref;
    int na;
    int64_t total;
};

// ---- device-side control of the batched refinement and cutoff search -------
// Largest Krylov dimension of a batched refinement.
constexpr int kMaxRestart = 38;
// Scalar slots of each problem (BProb::scal, doubles).
enum : int64_t {
    SC_RNORM = 0,   // ||b - Z x||_inf of the last residual evaluation
    SC_BETA = 1,    // ||M^{-1} r||_2
    SC_SUM = 2,     // sum, min, argmin of w (3)
    SC_AMAX = 5,    // ||b||_inf of a right-hand side
    SC_PICK = 6,    // an entry picked at a device index
    SC_H = 16,      // Arnoldi column h (2 (k+1)) and h_{k+1,k}
    SC_Y = 96,      // GMRES solution coefficients (kMaxRestart + 1)
    SC_RC = 136,    // refinement state (RC_* offsets)
    SC_HH = 160,    // Hessenberg matrix, column-major, (kMaxRestart + 1) x kMaxRestart
    SC_CS = SC_HH + (kMaxRestart + 1) * kMaxRestart,  // Givens cosines
    SC_SN = SC_CS + kMaxRestart,                      // Givens sines
    SC_G = SC_SN + kMaxRestart,                       // rotated right-hand side (kMaxRestart + 1)
    SC_COUNT = (SC_G + kMaxRestart + 1 + 63) / 64 * 64
};
enum : int { RC_RNORM = 0, RC_BEST, RC_PREV, RC_TOL, RC_BETA, RC_INNER, RC_KDONE, RC_ROUND };
// Control word of each problem (BProb::ints[kIntFlags]; status words and the
// preconditioner counters sit below it).
constexpr int kIntsPer = 2048;
constexpr int kIntFlags = kIntsPer - 8;
enum : int {
    F_SEARCH = 1 << 0,     // solved in this step
    F_REF = 1 << 1,        // refinement still running
    F_COPYBEST = 1 << 2,   // this round: x improved, copy it to the best iterate
    F_REVERT = 1 << 3,     // this round: back to the best iterate
    F_DOPLAIN = 1 << 4,    // this round: plain step x += M^{-1} r
    F_DOGMRES = 1 << 5,    // this round: a GMRES cycle
    F_INNER = 1 << 6,      // the GMRES cycle continues
    F_LASTPLAIN = 1 << 7,  // the last correction was a plain step
    F_PLAINMODE = 1 << 8,  // plain steps still gain two digits each
    F_REVERTED = 1 << 9,   // x was reset to the best iterate last round
    F_OK = 1 << 10,        // tol reached
    F_HI = 1 << 11,        // this step's w is the search's new upper bracket end
    F_NEEDD = 1 << 12,     // the search wants d(min w)/dt at this step's point
    F_BROKEN = 1 << 13     // the FP32 factor broke down (retaken with a shift)
};
// State of one cloud's cutoff search (device array, one thread per cloud).
// The rules are those of the single search: grid scan downward from the bound,
// then bisection in log t with safeguarded Newton steps, or Ridders' method.
struct SState {
    double tb, eps, top, hi, hi_min, lo, lo_min, last_t, last_min, last_d, prev_step, cur;
    double ra, rga, rb, rgb, rgm, shift;
    int32_t phase;       // 0 grid scan, 1 bracket refinement, 2 done; fixed-scale solves: 0 first, 2 done
    int32_t gi, ext, have_hi, have_lo, prev_newton, last_has_d, solves, newton_steps, no_sign;
    int32_t cur_newton, rid_pending, cur_kind, retry, attempts, err, unconverged, pad_;
};
struct SParams {
    int32_t grid, max_extend, newton, ridders, fixed;  // fixed: one solve per problem at BProb::t
    int32_t pad_;
    double lo_factor, rtol;
};

// FP64 kernel entry exp(-t d), d = sqrt(s), for the matrix-free products.
// sqrt_pos: square root of a normal s > 0 from the hardware reciprocal square
// root estimate, one Goldschmidt step (g ~ sqrt(s), h ~ 1/(2 sqrt(s))) and two
// FMA residual corrections g += (s - g^2) h (Markstein's scheme).
__device__ __forceinline__ double sqrt_pos(double s)
{
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double e = fma(-g, g, s);
    g = fma(e, h, g);
    e = fma(-g, g, s);
    return fma(e, h, g);
}

// a * b + c with a uniform c held in an SGPR pair: one VOP3 FMA (the compiler's
// two-address FMA form would copy a loop-invariant addend before every use)
__device__ __forceinline__ double fma_uc(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

// exp(x) for x <= 0: Cody-Waite reduction x = k ln2 + r with |r| <= ln2/2 (ln2
// split into a head with 32 significant bits, so k ln2_head is exact, and a
// tail), e^r from its Taylor series to degree 13 (truncation below 1e-17
// relative on that interval) in Horner form, then the exact scaling by 2^k,
// which underflows to 0 below about -745.
__device__ __forceinline__ double exp_nonpos(double x)
{
    x = fmax(x, -1.0e4);
    const double k = rint(x * 1.4426950408889634);  // log2(e)
    double r = fma(-k, 6.93147180369123816490e-01, x);
    r = fma(-k, 1.90821492927058770002e-10, r);
    double p = fma_uc(1.0 / 6227020800.0, r, 1.0 / 479001600.0);  // 1/13!, 1/12!
    p = fma_uc(p, r, 1.0 / 39916800.0);
    p = fma_uc(p, r, 1.0 / 3628800.0);
    p = fma_uc(p, r, 1.0 / 362880.0);
    p = fma_uc(p, r, 1.0 / 40320.0);
    p = fma_uc(p, r, 1.0 / 5040.0);
    p = fma_uc(p, r, 1.0 / 720.0);
    p = fma_uc(p, r, 1.0 / 120.0);
    p = fma_uc(p, r, 1.0 / 24.0);
    p = fma_uc(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// Z entry exp(-t sqrt(s)) for a squared distance s >= 0 (s = 0 gives 1); s is
// clamped into [1e-300, 1e300], where the entry is 1 and 0 to FP64
__device__ __forceinline__ double zexp(double t, double s)
{
    return exp_nonpos(-(t * sqrt_pos(fmin(fmax(s, 1.0e-300), 1.0e300))));
}

__device__ inline int bfind(const int64_t *pref, int na, int64_t u)
{
    int lo = 0, hi = na - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---- batched launchers (batch.hip drives them) ---------------------------------
int64_t tilegen32_blocks(int64_t npad);
void launch_tilegen32_b(hipStream_t s, const BProb *P, const BWork &w);
void launch_potrf128_b(hipStream_t s, const BProb *P, const BWork &w, int64_t k0);
int64_t gemm_b_units(int kind, int64_t npad, int64_t kk);
void launch_gemm_b(hipStream_t s, int kind, const BProb *P, const BWork &w, int64_t kk);
int64_t prec_b_units(int64_t npad);
void launch_prec_apply_b(hipStream_t s, const BProb *P, const BWork &w, int rhs_slot, int tmp_slot,
                         int x_slot);
int64_t zmv_b_units(int64_t n, int m);
int64_t zmv_b_reduce_units(int64_t n, int m);
void launch_zmv_b(hipStream_t s, int m, const BProb *P, const BWork &wz, const BWork &wr, int v_slot,
                  int y_slot, int b_slot, int mode, int64_t norm_off);
int64_t dz_b_units(int64_t n);
void launch_dzmv_b(hipStream_t s, int m, const BProb *P, const BWork &wz, const BWork &wr, int v_slot,
                   int y_slot);
void launch_fill_b(hipStream_t s, const BProb *P, const int *plist, int na, int64_t maxpad, int slot,
                   double v, bool upto_n);
void launch_copy_b(hipStream_t s, const BProb *P, const int *plist, int na, int64_t maxpad, int src, int dst);
void launch_scale_inv_b(hipStream_t s, const BProb *P, const int *plist, int na, int64_t maxpad, int src,
                        int dst, int64_t scal_off);
void launch_multidot_b(hipStream_t s, const BProb *P, const int *plist, int na, int v0, int k, int u_slot,
                       int64_t out_off);
void launch_multi_axpy_b(hipStream_t s, const BProb *P, const int *plist, int na, int64_t maxpad, int v0,
                         int k, int64_t h_off, int u_slot, double sign);
void launch_multi_axpy_hb(hipStream_t s, const BProb *P, const int *plist, int na, int64_t maxpad, int v0,
                          int k, const double *hb, int u_slot, double sign);
void launch_nrm2_b(hipStream_t s, const BProb *P, const int *plist, int na, int slot, int64_t out_off);
void launch_summin_b(hipStream_t s, const BProb *P, const int *plist, int na, int slot, int64_t out_off);
void launch_amax_b(hipStream_t s, const BProb *P, const int *plist, int na, int slot, int64_t out_off);
void launch_gather_scal_b(hipStream_t s, const BProb *P, const int *plist, int na, int64_t off, int cnt,
                          double *out);
void launch_pick_b(hipStream_t s, const BProb *P, const int *plist, int na, int slot, int64_t idx_off,
                   int64_t dst);
void launch_zero_status_b(hipStream_t s, const BProb *P, const int *plist, int na);

// ---- device-side control kernels (bctl.hip); problems are P[0..B) ----------
// active = ((flags & mask) == mask) for every problem
void launch_gate_b(hipStream_t s, BProb *P, int B, int mask);
// start a refinement for the active problems: F_REF set, tolerance
// tol * max(1, scal[bnorm_off]) (bnorm_off < 0: tol)
void launch_ref_init_b(hipStream_t s, BProb *P, int B, int64_t bnorm_off, double tol);
// decisions after a residual evaluation (see bctl.hip); final: no corrections
void launch_ref_decide_b(hipStream_t s, BProb *P, int B, int final_round, int max_gmres);
void launch_gmres_start_b(hipStream_t s, BProb *P, int B);
// Arnoldi step k on slots v0.. (V_{k+1} holds M^{-1} Z V_k): two classical
// Gram-Schmidt passes, norm, Givens rotation, the continue decision, scaling
void launch_arnoldi_b(hipStream_t s, BProb *P, int B, int k, int v0, int kcycle, double inner_tol,
                      int max_gmres);
void launch_gmres_finish_b(hipStream_t s, BProb *P, int B, int kcycle);
// x_slot += z_slot for the active problems
void launch_axpy_slot_b(hipStream_t s, BProb *P, int B, int64_t maxpad, int z_slot, int x_slot);
// cutoff search / fixed-scale solves
void launch_search_select_b(hipStream_t s, BProb *P, SState *S, int B, SParams prm);
void launch_breakdown_b(hipStream_t s, BProb *P, SState *S, int B);
void launch_search_update_b(hipStream_t s, BProb *P, SState *S, int B, SParams prm);
void launch_search_deriv_b(hipStream_t s, BProb *P, SState *S, int B);
// out[0] = clouds still searching, out[1] = any error
void launch_search_count_b(hipStream_t s, const SState *S, int B, int *out);
void launch_unpack_b(hipStream_t s, const BProb *P, const int *plist, int na, const int64_t *offs, int slot,
                     double *out, int64_t maxn);

}  // namespace mag

struct mag_ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    mag::DevBuf factor;    // FP32 npad^2 factor, or FP64 n^2 dense Z
    mag::DevBuf dinv;      // FP32 inverses of the 128-diagonal blocks
    mag::DevBuf vecs;      // FP64 vectors (Krylov basis and work vectors)
    mag::DevBuf partial;   // FP64 partial sums of split reductions
    mag::DevBuf ints;      // int32 counters / flags / status
    mag::DevBuf aux;       // FP64 vectors of the cutoff search and the adjoint
    // batched solves
    mag::DevBuf bfactor, bdinv, bvec, bscal, bpartial, bints, bdesc, barena, bstage;
    mag::DevBuf hodlr;     // HODLR preconditioner workspace
    mag::DevBuf eig;       // Lanczos bases of the eigenvalue estimator
    mag::DevBuf hss;       // HSS approximation and ULV factor
    void *bhost = nullptr;   // pinned host staging for work lists and descriptors
    size_t bhost_bytes = 0;
    double *host_scalars = nullptr;  // pinned host staging (64 doubles)
    void *blas = nullptr;            // rocblas_handle (lazy, FP64 comparator)
    int64_t cu_count = 256;
    // tuned panel width of the single-solve FP32 factor per size bucket
    // (bucket = bit length of npad); 0 = the built-in choice
    int tune_panel[64] = {};
    // tuned grouping of the batched factorisation's 256-column panels per size
    // bucket of the largest npad: 0 = built-in (pairs), 1 = single panels
    // (trailing updates with K = 256), 2 = pairs (K = 512)
    int tune_bgroup[64] = {};
    // cap on the device bytes held by the buffers above (0: none)
    size_t ws_limit = 0;
    // polls of one substitution wait before MAG_EINTERNAL (0: kSpinLimitDefault)
    int64_t spin_limit = 0;
};

namespace mag {

// Grow `b` to at least `bytes` (frees the old block; contents are lost).
// MAG_ENOMEM when the device cannot hold it or the context's cap would be
// exceeded.
int ensure(mag_ctx *ctx, DevBuf &b, size_t bytes);
// Device bytes held by the context's buffers.
size_t ctx_held_bytes(const mag_ctx *ctx);
// MAG_OK if `extra` more device bytes stay within the context's cap.
int ctx_may_allocate(const mag_ctx *ctx, size_t extra);
// Coordinates finite and pairwise distinct (else MAG_EINVAL / MAG_ENOTPD); one host sync.
// pairs = false checks finiteness only (the caller's FP32 tile generator checks the pairs).
int check_points(mag_ctx *ctx, const double *X, int64_t n, int m, bool pairs = true);

// Event pairs around the trailing-update launches of a factorisation, with
// the algorithmic flops of each launch.
struct FactorTimer {
    std::vector<hipEvent_t> ev;
    std::vector<double> flops;
    size_t used = 0;
};
// nb: panel width, 256 or 512 (npad is a multiple of 256)
void chol32_factor(hipStream_t s, float *A, int64_t npad, int64_t n, float *dinv, int *status,
                   FactorTimer *timer, int nb);
// panel width for npad on this context: the tuned entry of its size bucket, else 512
int panel_width(const mag_ctx *ctx, int64_t npad);
int size_bucket(int64_t npad);
size_t dmin_partial_doubles(int64_t n);
size_t blas1_partial_doubles(int kmax);

// pairwise.hip: derivative passes (matrix-free FP64)
int pair_max_dim();
size_t pair_partial_doubles(int64_t n, int m);
// y (npad) = (D o Z) v, i.e. -dZ/dt v
void launch_dzmv(hipStream_t s, const double *X, int64_t n, int m, double t, const double *v,
                 double *y, double *partial);
// dX (n x m) = t sum_{k != j} (lam_j w_k + lam_k w_j) Z_jk (x_j - x_k) / d_jk
void launch_gradx(hipStream_t s, const double *X, int64_t n, int m, double t, const double *w,
                  const double *lam, double *dX, double *partial);

// ---- launchers (all enqueue on ctx->stream) --------------------------------
// tilegen.hip
// status (optional): status[kStDuplicate] = 1 if some pair j != k < n has d_jk = 0.
// kernel kKernShiftDist writes t - d_jk (diagonal t + shift) instead of exp(-t d_jk).
void launch_tilegen32(hipStream_t s, const double *X, int64_t n, int m, double t,
                      float *A, int64_t npad, float shift, int *status = nullptr, int kernel = kKernExp);
void launch_tilegen64(hipStream_t s, const double *X, int64_t n, int m, double t, double *A);
// FP64 Z in the padded layout (npad x npad, lower triangle and the 128-diagonal
// tiles, identity padding); status[kStDuplicate] as launch_tilegen32.
void launch_tilegen64p(hipStream_t s, const double *X, int64_t n, int m, double t, double *A, int64_t npad,
                       int *status);
// Writes min squared distance partials; returns number of partials in *np.
void launch_dmin2(hipStream_t s, const double *X, int64_t n, int m, double *partial,
                  int64_t *np, double *out_min2);
void launch_check_finite(hipStream_t s, const double *X, int64_t count, int *status);

// gemm_mfma.hip: C (M x N) = [C] - P * Q^T (kGemmSub) or C = P * Q^T (kGemmSet),
// column-major operands: P is M x K (P[p*ldp + i]), Q is N x K (Q[p*ldq + j]).
// kGemmSetT also writes C^T to CT (CT(j, i) at CT[i * ldc + j]).
enum GemmMode { kGemmSub = 0, kGemmSet = 1, kGemmSetT = 2 };
// The panel path's contractions on 64-row x 128-column tiles: M a multiple of
// 64, N of 128, K of 16.  A workgroup owns whole 128-column row blocks of C, so
// C may alias P when N = 128 (the in-place panel solve).
void launch_gemm_rows64(hipStream_t s, float *C, int64_t ldc, const float *P, int64_t ldp, const float *Q,
                        int64_t ldq, int64_t M, int64_t N, int64_t K, GemmMode mode, float *CT = nullptr);
// C (N x N, lower 128-tiles only) -= P P^T with P N x K; N multiple of 128.
void launch_syrk_lower(hipStream_t s, float *C, int64_t ldc, const float *P, int64_t ldp,
                       int64_t N, int64_t K);

// gemm64.hip: the FP64 factor's contractions, C (M x N) -= P Q^T (kGemmSub) or
// C = P Q^T with C^T into CT (kGemmSetT); operands column-major as for
// launch_gemm_rows64.  tile 128: M, N multiples of 128, kGemmSub only; tile 64: M, N
// multiples of 64.  K a multiple of 16; operand pointers 16-byte aligned and
// leading dimensions even.
void launch_gemm64(hipStream_t s, int tile, double *C, int64_t ldc, const double *P, int64_t ldp, const double *Q,
                   int64_t ldq, int64_t M, int64_t N, int64_t K, GemmMode mode, double *CT);
// C (N x N, lower 128-tiles only) -= P P^T with P N x K; N multiple of 128.
void launch_syrk64_lower(hipStream_t s, double *C, int64_t ldc, const double *P, int64_t ldp, int64_t N, int64_t K);
// potrf64.hip: factor the 64 x 64 diagonal block at (k0, k0) of the FP64 A in
// place (L below and on the diagonal, L^T above) and write its inverse to Linv
// (64 x 64 column-major).  Breakdown -> status.
void launch_potrf64(hipStream_t s, double *A, int64_t ld, int64_t k0, double *Linv, int *status);
// chol64.hip: FP64 factor of the padded npad x npad A (layout of the FP32
// factor) in place; dinv receives the inverses of the 64-diagonal blocks
// (npad / 64 blocks of 64 x 64).
void chol64_factor(hipStream_t s, double *A, int64_t npad, int64_t n, double *dinv, int *status, FactorTimer *timer);

// potrf.hip: factor the 128 x 128 diagonal block at (k0, k0) of A in place and
// write its inverse to Linv (128 x 128 column-major).  Breakdown -> status.
void launch_potrf128(hipStream_t s, float *A, int64_t ld, int64_t k0, float *Linv, int *status);

// gemv64.hip: FP64 matrix-free products with Z regenerated from X.
//   mode 0: y = Z v;  mode 1: y = b - Z v (b may be NULL meaning ones) and
//   out_norm[0] = ||y||_inf (device scalar).
//   f32_entries: each entry exp(-t d) evaluated in FP32 (sums stay FP64); the
//   inner products of GMRES may take it, residuals never do (m <= 16 only).
//   kernel: kKernExp the entries exp(-t d) of Z; kKernShiftDist the entries
//   t - d of the scale-zero system c 1 1^T - d with c passed as t (m <= 16).
void launch_zmv(hipStream_t s, const double *X, int64_t n, int m, double t,
                const double *v, double *y, const double *b, int mode,
                double *partial, double *out_norm, bool f32_entries = false, int kernel = kKernExp);
size_t zmv_partial_doubles(int64_t n);
// The row-per-thread form of launch_zmv (any m; no symmetric tiles): partial
// needs zmv_split_partial_doubles(n) doubles, y npad doubles; the max norm of
// mode 1 goes to out_norm (may be NULL).
void launch_zmv_split(hipStream_t s, const double *X, int64_t n, int m, double t, const double *v,
                      double *y, const double *b, int mode, double *partial, double *out_norm);
size_t zmv_split_partial_doubles(int64_t n);
// Per-device address of the no-allocation entry point's scratch array, taken
// once per device (with that device current) by mag_create.
int noalloc_setup(int device);

// Polls of one wait of the sync-free substitutions before they give up and
// report MAG_EINTERNAL (mag_set_spin_limit overrides it per context).
constexpr long kSpinLimitDefault = 1L << 26;
// trsv.hip: z = L^{-T} L^{-1} r with the FP32 factor, FP64 arithmetic, by the
// one-block-per-workgroup substitution with a composite near step.  Q: the near
// tiles of launch_near_q for this factor (required).
void launch_prec_apply(hipStream_t s, const float *L, int64_t npad, const float *dinv,
                       const double *r, double *y_tmp, double *z, int *counters, int *status,
                       const float *Q, long spin_limit);
// The near tiles D_b T(b, b -/+ 1) of every 128-block of the FP32 factor, both
// directions (near_q_floats(npad) floats), from the factor and its inverses.
size_t near_q_floats(int64_t npad);
void launch_near_q(hipStream_t s, const float *A, int64_t npad, const float *dinv, float *Q);
size_t prec_counter_ints();
// z = L^{-T} L^{-1} r with the FP64 factor of chol64_factor (64-blocks).
void launch_chol64_solve(hipStream_t s, const double *L, int64_t npad, const double *dinv, const double *r,
                         double *y_tmp, double *z, int *counters, int *status,
                         long spin_limit);

// blas1.hip: deterministic FP64 vector kernels (length npad, two-pass).
void launch_fill(hipStream_t s, double *x, int64_t len, double v);
void launch_fill_ints(hipStream_t s, int *x, int64_t len, int v);
void launch_copy(hipStream_t s, const double *x, double *y, int64_t len);
// h[i] = V_i . u for i < k (V rows of stride ld), result in device h (k doubles).
void launch_multidot(hipStream_t s, const double *V, int64_t ld, int k, const double *u,
                     int64_t len, double *partial, double *h);
// u -= sum_i h[i] V_i
void launch_multi_axpy(hipStream_t s, const double *V, int64_t ld, int k, const double *h,
                       double *u, int64_t len, double sign);
// out = ||x||_2 (device scalar)
void launch_nrm2(hipStream_t s, const double *x, int64_t len, double *partial, double *out);
// y = x * (1/alpha[0]) with device alpha
void launch_scale_inv(hipStream_t s, const double *x, double *y, int64_t len, const double *alpha);
// y += x
void launch_axpy1(hipStream_t s, const double *x, double *y, int64_t len);
// sum (block sums combined with Neumaier compensation), min, argmin of x[0..n):
// out[0]=sum, out[1]=min, out[2]=argmin
void launch_sum_min(hipStream_t s, const double *x, int64_t n, double *partial, double *out);
// out = max |x_i|
void launch_amax(hipStream_t s, const double *x, int64_t len, double *partial, double *out);
// y = a*1 + x on [0, n) (x may be NULL), zero on [n, len)
void launch_affine_ones(hipStream_t s, const double *x, double a, double *y, int64_t n, int64_t len);
// y = a*x on [0, n), zero on [n, len)
void launch_scale(hipStream_t s, const double *x, double a, double *y, int64_t n, int64_t len);
// y_j = 1/2 + frac((j + 1) g), g = (sqrt 5 - 1)/2, on [0, n); zero on [n, len)
void launch_golden(hipStream_t s, double *y, int64_t n, int64_t len);

// ---- hodlr.hip: HODLR preconditioner ---------------------------------------------
// Device pointers into ctx->hodlr (valid until the next HODLR factorisation on
// the same context).  Points are in tree order (perm[i] = caller index of the
// i-th point); node (l, i) covers [bnd[2^l - 1 + l + i], ... + 1).  Level l's
// bases have k[l] columns (a multiple of 64) at P + poff[l] / Ph + poff[l];
// its nodes' [B | C | S^{-1}] blocks (k[l] x k[l] each) start at W + woff[l].
struct HodlrFactor {
    int64_t n = 0, npad = 0;
    int m = 0, L = 0, ls = 0;  // ls: leaf storage stride (ls x ls inverse per leaf)
    double t = 0.0;
    double *Xp = nullptr, *P = nullptr, *Ph = nullptr, *Dinv = nullptr, *W = nullptr;
    double *apart = nullptr, *tv = nullptr, *xp = nullptr;
    int64_t *perm = nullptr, *bnd = nullptr;
    std::vector<int64_t> bnd_host, poff, woff, csz;
    std::vector<int> k, crows, cmax;
};
// Ridders' point for the bracket s_a < s_b with g_a < 0 <= g_b, from g_m at the
// midpoint: s_m + (s_m - s_a) sign(g_a - g_b) g_m / sqrt(g_m^2 - g_a g_b).  It lies
// in [s_a, s_b] since g_m^2 - g_a g_b >= g_m^2; the midpoint when undefined.
__host__ __device__ inline double ridders_point(double sa, double ga, double sb, double gb, double gm)
{
    const double sm = 0.5 * (sa + sb);
    const double den = sqrt(gm * gm - ga * gb);
    if (!(den > 0.0) || !(den < INFINITY)) return sm;
    const double sgn = (ga - gb) < 0.0 ? -1.0 : 1.0;
    const double sx = sm + (sm - sa) * sgn * gm / den;
    return fmin(fmax(sx, sa), sb);
}

int hodlr_max_leaf();
int hodlr_default_leaf();
int hodlr_max_cols();
int hodlr_levels(int64_t n, int leaf);
// Build the factor of Z(t) for the points X (device, n x m); rank0 is the
// basis rank of the top level (halved every two levels), oversample the extra
// sample columns, power the subspace iterations of the range finder.  Status
// words in ctx->ints.  MAG_ENOTPD when a leaf block is not positive definite.
int hodlr_factor(mag_ctx *ctx, const double *X, int64_t n, int m, double t, int leaf, int rank0,
                 int oversample, int power, uint64_t seed, HodlrFactor &H);
// z = H^{-1} r; r, z device vectors of length npad (z zero on [n, npad)).
void hodlr_apply(hipStream_t s, const HodlrFactor &H, const double *r, double *z);

// ---- hodlr.hip: HSS approximation with nested bases and its ULV factor --------
// Same cluster tree as the HODLR (points in tree order, perfect tree of L
// levels).  Level l (1 <= l <= L) has 2^l nodes with a[l] active unknowns each
// (the leaf size ell at l = L, else the two children's k[l+1]) and orthogonal
// Q (a x a, column-major) whose last k[l] columns are the node's basis; level
// 0 is the root, a dense block of a[0] = 2 k[1] unknowns.  Dt holds, per node,
// the transformed block Q^T D Q after elimination: L_e^{-1} (the inverse of the
// Cholesky factor L_e of the first e = a - k unknowns, lower triangle)
// top-left, W = D_se L_e^{-T} bottom-left and the Schur complement passed to
// the parent bottom-right.  Root: Cholesky of its
// block.  ub/xb: per-level work vectors of the apply.
struct HssFactor {
    int64_t n = 0, npad = 0;
    int m = 0, L = 0, ell = 0;
    double t = 0.0;
    double *Xp = nullptr, *Q = nullptr, *Dt = nullptr, *Droot = nullptr, *ub = nullptr, *xb = nullptr;
    double *xl = nullptr, *rr = nullptr;
    double *tv = nullptr, *part = nullptr;  // the apply's temporary vector and partial sums
    int64_t *perm = nullptr, *bnd = nullptr;
    std::vector<int> k, a;
    std::vector<int64_t> off;  // per level: offset of its Q / Dt blocks (doubles)
    std::vector<int64_t> voff; // per level: offset of its ub / xb vectors (doubles)
    void *blas = nullptr;      // rocblas_handle of the context
    double shift = 0.0;        // largest diagonal shift a compressed block needed (0: none)
};
// Build the HSS approximation of Z(t) (ranks from rank0 and oversample as
// documented for mag_opts.max_rank) and its ULV factor.  MAG_ENOTPD when a
// block to be eliminated is not positive definite.
int hss_factor(mag_ctx *ctx, const double *X, int64_t n, int m, double t, int leaf, int rank0, int oversample,
               uint64_t seed, HssFactor &H);
// z = H^{-1} r (npad vectors, caller's point order; z zero on [n, npad)).
int hss_apply(hipStream_t s, const HssFactor &H, const double *r, double *z);

}  // namespace mag
