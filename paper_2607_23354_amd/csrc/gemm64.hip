// gemm64.hip -- FP64 MFMA kernels of the FP64 blocked Cholesky.
//
//   C (M x N)  <-  C - P Q^T      (kGemmSub: trailing SYRK/GEMM updates)
//   C (M x N)  <-  P Q^T          (kGemmSetT: panel TRSM against an explicit
//                                   inverse of the diagonal block, with C^T
//                                   also written to CT, CT(j, i) = CT[i * ldc + j])
//
// The FP64 factor is the dense comparator of the FP32 + refinement solve: the
// same blocked right-looking Cholesky of Z (symmetric positive definite for
// distinct Euclidean points, Section 3.2), in FP64 throughout.  Operands are
// column-major FP64: P(i, p) = P[p * ldp + i], Q(j, p) = Q[p * ldq + j],
// C(i, j) = C[j * ldc + i].
//
// Matrix cores: v_mfma_f64_16x16x4f64, D (16 x 16) += A (16 x 4) B (4 x 16).
// Lane l = 16 kq + q supplies A(q, kq) and B(kq, q), and holds
// D(kq + 4 v, q) in register v.  A is taken from Q and B from P, so
// D(r, c) = (P Q^T)(i0 + c, j0 + r): the 16 lanes of one kq hold 16
// consecutive rows of one column of C, a 128-byte line.
//
// Workgroup tile BM x BN (128 x 128 for the trailing updates, 64 x 64 for the
// panel's short-K products), 4 waves in a 2 x 2 arrangement, each wave a
// (BM/2) x (BN/2) sub-tile of 16 x 16 MFMA blocks.  K is staged through LDS
// by direct global-to-LDS loads: the long-K updates in chunks of 16,
// double-buffered, one barrier per stage; the panel's K = 64 products in one
// stage (all loads in flight at once: these launches are latency bound).  A
// 128-wide stage row is padded to 144 doubles, so the four k-rows one MFMA
// operand read touches fall on disjoint bank halves.
#include "internal.hpp"

namespace mag {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) void *gptr;  // global operand of a direct LDS load
typedef __attribute__((address_space(3))) void *lptr;        // its LDS destination

constexpr int KC = 16;   // K per LDS stage of the long-K updates
constexpr int KP = 64;   // K of the panel's products (one stage)
constexpr int NT = 256;  // threads per workgroup
constexpr int kXcds = 8;

// row stride (doubles) of a stage row of B entries
template <int B>
constexpr int stage_ld() { return B == 128 ? 144 : B; }

template <int BM, int BN, int MODE, int KS, int NBUF>
constexpr int lds_doubles()
{
    // NBUF buffers of P and Q stages; the SetT epilogue's transposed tile reuses them
    constexpr int st = NBUF * KS * (stage_ld<BM>() + stage_ld<BN>());
    constexpr int tr = (MODE == kGemmSetT) ? BN * (BM + 1) : 0;
    return st > tr ? st : tr;
}

__device__ inline void tri_index(int64_t idx, int64_t &ti, int64_t &tj)
{
    int64_t r = (int64_t)((sqrt(8.0 * (double)idx + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > idx) --r;
    while ((r + 1) * (r + 2) / 2 <= idx) ++r;
    ti = r;
    tj = idx - r * (r + 1) / 2;
}

// Stage KS rows of B entries (a column-major operand X, rows x0.., k = k0..)
// into S (row stride stage_ld<B>()) by direct loads: one wave instruction moves
// 64 x 16 bytes, a 128-entry row or two 64-entry rows; wave w moves rows
// [w KS/4, (w + 1) KS/4).
template <int B, int KS>
__device__ __forceinline__ void stage_rows(const double *X, int64_t ldx, int64_t x0, double *S, int wave, int lane)
{
    constexpr int SL = stage_ld<B>();
    if constexpr (B == 128) {
#pragma unroll
        for (int u = 0; u < KS / 4; ++u) {
            const int p = wave * (KS / 4) + u;
            __builtin_amdgcn_global_load_lds((gptr)(X + (int64_t)p * ldx + x0 + 2 * lane), (lptr)(S + p * SL), 16, 0,
                                             0);
        }
    } else {
        static_assert(B == 64, "tile edge 64 or 128");
#pragma unroll
        for (int u = 0; u < KS / 8; ++u) {
            const int p = 2 * (wave * (KS / 8) + u);
            __builtin_amdgcn_global_load_lds((gptr)(X + (int64_t)(p + (lane >> 5)) * ldx + x0 + 2 * (lane & 31)),
                                             (lptr)(S + p * SL), 16, 0, 0);
        }
    }
}

// KS: K per stage; NBUF = 2 double-buffers stages of a long K, NBUF = 1 takes
// K = KS in one stage.
template <int BM, int BN, int MODE, int KS = KC, int NBUF = 2>
__device__ __forceinline__ void gemm64_tile(double *__restrict__ C, int64_t ldc, const double *__restrict__ P,
                                            int64_t ldp, const double *__restrict__ Q, int64_t ldq, int64_t ti,
                                            int64_t tj, int64_t K, double *__restrict__ CT)
{
    static_assert(MODE == kGemmSub || MODE == kGemmSetT, "modes of the FP64 factor");
    constexpr int SM = stage_ld<BM>(), SN = stage_ld<BN>();
    constexpr int MI = BM / 32, MJ = BN / 32;  // 16 x 16 blocks per wave in i and j
    __shared__ double lds[lds_doubles<BM, BN, MODE, KS, NBUF>()];
    double *Ps = lds;                     // [NBUF][KS][SM]
    double *Qs = lds + NBUF * KS * SM;    // [NBUF][KS][SN]
    const int64_t i0 = ti * BM, j0 = tj * BN;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wi = (wave & 1) * (BM / 2);
    const int wj = (wave >> 1) * (BN / 2);
    const int q = lane & 15, kq = lane >> 4;

    v4d acc[MI][MJ];
#pragma unroll
    for (int ib = 0; ib < MI; ++ib)
#pragma unroll
        for (int jb = 0; jb < MJ; ++jb) acc[ib][jb] = v4d{0.0, 0.0, 0.0, 0.0};

    // a one-stage update reads its C tile at once too, so every load of the
    // workgroup is in flight before the first wait
    constexpr bool kPreC = MODE == kGemmSub && NBUF == 1;
    double cpre[kPreC ? MI : 1][kPreC ? MJ : 1][4];
    if constexpr (kPreC) {
#pragma unroll
        for (int ib = 0; ib < MI; ++ib)
#pragma unroll
            for (int jb = 0; jb < MJ; ++jb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    cpre[ib][jb][v] = C[(j0 + wj + 16 * jb + kq + 4 * v) * ldc + i0 + wi + 16 * ib + q];
    }
    stage_rows<BM, KS>(P, ldp, i0, Ps, wave, lane);
    stage_rows<BN, KS>(Q, ldq, j0, Qs, wave, lane);
    __syncthreads();
    const int nst = (NBUF == 1) ? 1 : (int)(K / KS);
    for (int st = 0; st < nst; ++st) {
        const int buf = (NBUF == 1) ? 0 : (st & 1);
        if (NBUF > 1 && st + 1 < nst) {
            // the other buffer was last read before the previous barrier
            const int64_t k1 = (int64_t)(st + 1) * KS;
            stage_rows<BM, KS>(P + k1 * ldp, ldp, i0, Ps + (buf ^ 1) * KS * SM, wave, lane);
            stage_rows<BN, KS>(Q + k1 * ldq, ldq, j0, Qs + (buf ^ 1) * KS * SN, wave, lane);
        }
        const double *pb = Ps + buf * KS * SM + kq * SM + wi + q;
        const double *qb = Qs + buf * KS * SN + kq * SN + wj + q;
#pragma unroll
        for (int kk = 0; kk < KS / 4; ++kk) {
            double av[MJ], bv[MI];
#pragma unroll
            for (int jb = 0; jb < MJ; ++jb) av[jb] = qb[4 * kk * SN + 16 * jb];
#pragma unroll
            for (int ib = 0; ib < MI; ++ib) bv[ib] = pb[4 * kk * SM + 16 * ib];
#pragma unroll
            for (int ib = 0; ib < MI; ++ib)
#pragma unroll
                for (int jb = 0; jb < MJ; ++jb)
                    acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[jb], bv[ib], acc[ib][jb], 0, 0, 0);
        }
        __syncthreads();  // waits for the direct loads of the next stage too
    }

    // C(i, j) with i = i0 + wi + 16 ib + q, j = j0 + wj + 16 jb + kq + 4 v
#pragma unroll
    for (int ib = 0; ib < MI; ++ib) {
        const int64_t i = i0 + wi + 16 * ib + q;
#pragma unroll
        for (int jb = 0; jb < MJ; ++jb) {
            double *cp = C + (j0 + wj + 16 * jb + kq) * ldc + i;
            if (MODE == kGemmSub) {
                double cv[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) cv[v] = kPreC ? cpre[kPreC ? ib : 0][kPreC ? jb : 0][v] : cp[4 * v * ldc];
#pragma unroll
                for (int v = 0; v < 4; ++v) cp[4 * v * ldc] = cv[v] - acc[ib][jb][v];
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) cp[4 * v * ldc] = acc[ib][jb][v];
            }
        }
    }
    if (MODE == kGemmSetT) {
        // transposed copy through LDS (free after the last stage's barrier):
        // T[jl * (BM + 1) + il], then rows of CT written with consecutive j
        double *T = lds;
#pragma unroll
        for (int ib = 0; ib < MI; ++ib)
#pragma unroll
            for (int jb = 0; jb < MJ; ++jb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    T[(wj + 16 * jb + kq + 4 * v) * (BM + 1) + wi + 16 * ib + q] = acc[ib][jb][v];
        __syncthreads();
        static_assert(NT % BN == 0, "whole rows of CT per pass");
        const int jl = threadIdx.x % BN;
        for (int il = threadIdx.x / BN; il < BM; il += NT / BN)
            CT[(i0 + il) * ldc + j0 + jl] = T[jl * (BM + 1) + il];
    }
}

template <int BM, int BN, int MODE, int KS, int NBUF>
__global__ void __launch_bounds__(NT, 2)
k_gemm64(double *__restrict__ C, int64_t ldc, const double *__restrict__ P, int64_t ldp,
         const double *__restrict__ Q, int64_t ldq, int64_t tilesM, int64_t K, double *__restrict__ CT)
{
    gemm64_tile<BM, BN, MODE, KS, NBUF>(C, ldc, P, ldp, Q, ldq, blockIdx.x % tilesM, blockIdx.x / tilesM, K, CT);
}

// Trailing symmetric update C -= P P^T on the lower 128-tiles of C only, in
// the XCD-aware order of the FP32 factor's update: workgroups are dealt to the
// 8 XCDs round-robin by id, and consecutive ids of one XCD walk the se x se
// tiles of one super-tile of the lower triangle, whose 2 se operand panels
// (2 se x 128 rows x K doubles: 4 MB at se = 4, K = 512) stay in that XCD's L2.
__global__ void __launch_bounds__(NT, 2)
k_syrk64_lower(double *__restrict__ C, int64_t ldc, const double *__restrict__ P, int64_t ldp, int64_t tilesM,
               int64_t K, int se)
{
    const int64_t b = blockIdx.x;
    const int64_t xcd = b % kXcds, slot = b / kXcds;
    const int64_t sidx = (slot / (se * se)) * kXcds + xcd, within = slot % (se * se);
    int64_t si, sj;
    tri_index(sidx, si, sj);
    const int64_t ti = si * se + within / se;
    const int64_t tj = sj * se + within % se;
    if (tj > ti || ti >= tilesM) return;  // padding slot (uniform per workgroup)
    gemm64_tile<128, 128, kGemmSub, KC, 2>(C, ldc, P, ldp, P, ldp, ti, tj, K, nullptr);
}

}  // namespace

void launch_gemm64(hipStream_t s, int tile, double *C, int64_t ldc, const double *P, int64_t ldp, const double *Q,
                   int64_t ldq, int64_t M, int64_t N, int64_t K, GemmMode mode, double *CT)
{
    const int64_t tm = M / tile, tn = N / tile;
    if (tm <= 0 || tn <= 0 || K <= 0) return;
    const dim3 g((unsigned)(tm * tn));
    if (tile == 128)
        hipLaunchKernelGGL((k_gemm64<128, 128, kGemmSub, KC, 2>), g, dim3(NT), 0, s, C, ldc, P, ldp, Q, ldq, tm, K,
                           CT);
    else if (K != KP)  // a 64-tile product of another depth: double-buffered stages
        hipLaunchKernelGGL((k_gemm64<64, 64, kGemmSub, KC, 2>), g, dim3(NT), 0, s, C, ldc, P, ldp, Q, ldq, tm, K, CT);
    else if (mode == kGemmSub)
        hipLaunchKernelGGL((k_gemm64<64, 64, kGemmSub, KP, 1>), g, dim3(NT), 0, s, C, ldc, P, ldp, Q, ldq, tm, K, CT);
    else
        hipLaunchKernelGGL((k_gemm64<64, 64, kGemmSetT, KP, 1>), g, dim3(NT), 0, s, C, ldc, P, ldp, Q, ldq, tm, K,
                           CT);
}

void launch_syrk64_lower(hipStream_t s, double *C, int64_t ldc, const double *P, int64_t ldp, int64_t N, int64_t K)
{
    const int64_t tm = N / 128;
    if (tm <= 0 || K <= 0) return;
    const int se = 4;
    const int64_t st = (tm + se - 1) / se;
    const int64_t nsup = st * (st + 1) / 2;
    const int64_t blocks = ((nsup + kXcds - 1) / kXcds) * kXcds * se * se;
    hipLaunchKernelGGL(k_syrk64_lower, dim3((unsigned)blocks), dim3(NT), 0, s, C, ldc, P, ldp, tm, K, se);
}

}  // namespace mag
