// potrf.hip -- Cholesky factor and inverse of one 128 x 128 diagonal block.
//
// The blocked right-looking Cholesky (factor of Z, which is symmetric
// positive definite for distinct Euclidean points, Section 3.2) needs at each
// panel step the factor L11 of the diagonal block and, to turn the panel's
// triangular solve into an MFMA contraction, the explicit inverse L11^{-1}.
// Both are computed here by a single workgroup with the block held in LDS:
//
//   for each 32-column block J (right-looking):
//     1. one wave factors the 32 x 32 diagonal block in registers
//        (lane = row, pivots and columns broadcast with readlane) and
//        inverts it by substitution;
//     2. the blocks below are solved against it, L_IJ = A_IJ inv(L_JJ)^T;
//     3. the trailing blocks are updated, A_IK -= L_IJ L_KJ^T;
//   then the off-diagonal blocks of the inverse, by distance from the
//   diagonal: Inv_IJ = -Inv_II sum_{K=J}^{I-1} L_IK Inv_KJ.
// Steps 2, 3 and the inverse are 32 x 32 x 32 products on MFMA
// (v_mfma_f32_32x32x2f32, one product per wave).
//
// A pivot that is not positive (or not finite) marks status[0] with the
// global pivot index + 1 and is replaced by 1 so the kernel still finishes;
// the host then refactors with a diagonal shift.
#include "internal.hpp"

namespace mag {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int NB = 128;
constexpr int LDS_LD = 129;  // padded column stride of the LDS copy
constexpr int TLD = 33;

__device__ inline float bcast(float v, int src_lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src_lane));
}

// acc += X Y for 32 x 32 blocks in column-major LDS (X(i, k) = X[k * xld + i]).
// YT: Y is given transposed, Y(k, j) = Yb(j, k); else Y(k, j) = Yb[j * yld + k].
// Accumulator lane l holds column-of-X-rows i = l % 32; register r holds
// j = 8 (r / 4) + 4 (l / 32) + r % 4.
template <bool YT>
__device__ inline v16f blk_mma(const float *X, int xld, const float *Yb, int yld, v16f acc, int lane)
{
    const int q = lane & 31, kq = lane >> 5;
#pragma unroll
    for (int kk = 0; kk < 32; kk += 2) {
        const float aop = YT ? Yb[(kk + kq) * yld + q] : Yb[q * yld + kk + kq];
        const float bop = X[(kk + kq) * xld + q];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(aop, bop, acc, 0, 0, 0);
    }
    return acc;
}

// dst(i, j) = (accumulate ? dst(i, j) : 0) + sign * acc for a 32 x 32 block
__device__ inline void blk_store(float *dst, int ld, const v16f &acc, int lane, float sign, bool accumulate)
{
    const int i = lane & 31, hi = lane >> 5;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int j = 8 * (r >> 2) + 4 * hi + (r & 3);
        float *p = dst + j * ld + i;
        *p = accumulate ? (*p + sign * acc[r]) : sign * acc[r];
    }
}

__device__ inline v16f zero16()
{
    v16f z;
#pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = 0.0f;
    return z;
}

__device__ __forceinline__ void potrf128_body(float *__restrict__ A, int64_t ld, int64_t k0,
                                              float *__restrict__ Linv, int *__restrict__ status)
{
    __shared__ float S[NB * LDS_LD];    // L, column-major, S[c*LDS_LD + r]
    __shared__ float V[NB * LDS_LD];    // L^{-1}, same layout
    __shared__ float T[3 * 32 * TLD];   // per-wave scratch for the off-diagonal inverse blocks
    __shared__ int bad;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    float *Ablk = A + k0 * ld + k0;

    // 16 float4 loads per thread, all in flight before the first LDS store
    {
        float4 buf[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e4 = tid + 256 * i;
            const int c = e4 >> 5, r4 = (e4 & 31) * 4;
            buf[i] = *reinterpret_cast<const float4 *>(Ablk + (int64_t)c * ld + r4);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e4 = tid + 256 * i;
            const int c = e4 >> 5, r4 = (e4 & 31) * 4;
            float *dst = S + c * LDS_LD + r4;
            dst[0] = buf[i].x;
            dst[1] = buf[i].y;
            dst[2] = buf[i].z;
            dst[3] = buf[i].w;
        }
    }
    if (tid == 0) bad = 0;
    __syncthreads();

    for (int J = 0; J < 4; ++J) {
        const int j0 = 32 * J;
        // 1. factor and invert the diagonal 32 x 32 block in wave 0 (lanes 32..63 mirror 0..31)
        if (wave == 0) {
            const int rr = lane & 31;
            float a[32];
#pragma unroll
            for (int c = 0; c < 32; ++c) a[c] = S[(j0 + c) * LDS_LD + j0 + rr];
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                float piv = bcast(a[c], c);
                if (!(piv > 0.0f) || !isfinite(piv)) {
                    if (lane == 0 && bad == 0) bad = (int)(k0 + j0 + c + 1);
                    piv = 1.0f;
                }
                const float inv = rsqrtf(piv);
                if (rr == c) a[c] = piv * inv;
                else if (rr > c) a[c] = a[c] * inv;
#pragma unroll
                for (int k = c + 1; k < 32; ++k) {
                    const float lkc = bcast(a[c], k);
                    if (rr >= k) a[k] = a[k] - a[c] * lkc;
                }
            }
            if (lane < 32) {
#pragma unroll
                for (int c = 0; c < 32; ++c)
                    if (c <= rr) S[(j0 + c) * LDS_LD + j0 + rr] = a[c];
            }
            // inverse of L_JJ by substitution, lane jc = column (rows i < jc stay 0)
            const int jc = lane & 31;
            float x[32];
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                float v = (i == jc) ? 1.0f : 0.0f;
#pragma unroll
                for (int k = 0; k < i; ++k) v = v - S[(j0 + k) * LDS_LD + j0 + i] * x[k];
                x[i] = v * __builtin_amdgcn_rcpf(S[(j0 + i) * LDS_LD + j0 + i]);
            }
            if (lane < 32) {
#pragma unroll
                for (int i = 0; i < 32; ++i) V[(j0 + jc) * LDS_LD + j0 + i] = x[i];
            }
        }
        __syncthreads();
        // 2. blocks below: L_IJ = A_IJ inv(L_JJ)^T, one block per wave
        {
            const int I = J + 1 + wave;
            if (I < 4) {
                v16f acc = blk_mma<true>(S + j0 * LDS_LD + 32 * I, LDS_LD, V + j0 * LDS_LD + j0, LDS_LD,
                                         zero16(), lane);
                blk_store(S + j0 * LDS_LD + 32 * I, LDS_LD, acc, lane, 1.0f, false);
            }
        }
        __syncthreads();
        // 3. trailing blocks (I, K), J < K <= I: A_IK -= L_IJ L_KJ^T
        {
            const int rem = 3 - J;                 // block rows below J
            const int npair = rem * (rem + 1) / 2;
            for (int pidx = wave; pidx < npair; pidx += 4) {
                int Kr = 0;
                while ((Kr + 1) * (Kr + 2) / 2 <= pidx) ++Kr;  // pidx -> (Ir >= Kr) pairs
                const int Ir = Kr, Kc = pidx - Kr * (Kr + 1) / 2;
                const int I = J + 1 + Ir, K = J + 1 + Kc;
                v16f acc = blk_mma<true>(S + j0 * LDS_LD + 32 * I, LDS_LD, S + j0 * LDS_LD + 32 * K, LDS_LD,
                                         zero16(), lane);
                blk_store(S + (32 * K) * LDS_LD + 32 * I, LDS_LD, acc, lane, -1.0f, true);
            }
        }
        __syncthreads();
    }

    // write L back (lower triangle including the diagonal) and L^T above it
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        const int e4 = tid + 256 * i;
        const int c = e4 >> 5, r4 = (e4 & 31) * 4;
        float4 v;
        v.x = (r4 + 0 >= c) ? S[c * LDS_LD + r4 + 0] : S[(r4 + 0) * LDS_LD + c];
        v.y = (r4 + 1 >= c) ? S[c * LDS_LD + r4 + 1] : S[(r4 + 1) * LDS_LD + c];
        v.z = (r4 + 2 >= c) ? S[c * LDS_LD + r4 + 2] : S[(r4 + 2) * LDS_LD + c];
        v.w = (r4 + 3 >= c) ? S[c * LDS_LD + r4 + 3] : S[(r4 + 3) * LDS_LD + c];
        *reinterpret_cast<float4 *>(Ablk + (int64_t)c * ld + r4) = v;
    }

    // off-diagonal blocks of the inverse by distance d = I - J (one block per wave)
    for (int d = 1; d < 4; ++d) {
        const int J = wave, I = J + d;
        if (I < 4) {
            float *Tw = T + wave * 32 * TLD;
            v16f acc = zero16();
            for (int K = J; K < I; ++K)
                acc = blk_mma<false>(S + (32 * K) * LDS_LD + 32 * I, LDS_LD, V + (32 * J) * LDS_LD + 32 * K,
                                     LDS_LD, acc, lane);
            blk_store(Tw, TLD, acc, lane, 1.0f, false);
            v16f acc2 = blk_mma<false>(V + (32 * I) * LDS_LD + 32 * I, LDS_LD, Tw, TLD, zero16(), lane);
            blk_store(V + (32 * J) * LDS_LD + 32 * I, LDS_LD, acc2, lane, -1.0f, false);
        }
        __syncthreads();
    }
    for (int e = tid; e < NB * NB; e += 256) {
        const int r = e & (NB - 1), c = e >> 7;
        Linv[c * NB + r] = (r >= c) ? V[c * LDS_LD + r] : 0.0f;
    }
    if (tid == 0 && bad != 0) atomicCAS(&status[kStBreakdown], 0, bad);
}

__global__ void __launch_bounds__(256)
k_potrf128(float *__restrict__ A, int64_t ld, int64_t k0, float *__restrict__ Linv,
           int *__restrict__ status)
{
    potrf128_body(A, ld, k0, Linv, status);
}

// Batched: one workgroup per problem whose padded size exceeds k0.
__global__ void __launch_bounds__(256)
k_potrf128_b(const BProb *__restrict__ P, BWork w, int64_t k0)
{
    const BProb &q = P[w.plist[blockIdx.x]];
    if (!q.active || k0 >= q.npad) return;
    potrf128_body(q.A, q.npad, k0, q.dinv + (k0 / NB) * NB * NB, q.ints);
}

}  // namespace

void launch_potrf128_b(hipStream_t s, const BProb *P, const BWork &w, int64_t k0)
{
    if (w.na > 0) hipLaunchKernelGGL(k_potrf128_b, dim3(w.na), dim3(256), 0, s, P, w, k0);
}

void launch_potrf128(hipStream_t s, float *A, int64_t ld, int64_t k0, float *Linv, int *status)
{
    hipLaunchKernelGGL(k_potrf128, dim3(1), dim3(256), 0, s, A, ld, k0, Linv, status);
}

}  // namespace mag
