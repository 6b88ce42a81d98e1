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
//        (lane = row, pivot and columns broadcast with readlane);
//     2. rows below it are solved against L_JJ^T (one thread per row);
//     3. the trailing part of the block is updated (4 x 4 register blocks).
//   then the inverse: diagonal 32 x 32 blocks by substitution (one wave
//   each), off-diagonal blocks by Inv_IJ = -Inv_II sum_{K=J}^{I-1} L_IK Inv_KJ.
//
// A pivot that is not positive (or not finite) marks status[0] with the
// global pivot index + 1 and is replaced by 1 so the kernel still finishes;
// the host then refactors with a diagonal shift.
#include "internal.hpp"

namespace mag {
namespace {

constexpr int NB = 128;
constexpr int LDS_LD = 129;  // padded column stride of the LDS copy
constexpr int TLD = 33;

__device__ inline float bcast(float v, int src_lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src_lane));
}

__device__ __forceinline__ void potrf128_body(float *__restrict__ A, int64_t ld, int64_t k0,
                                              float *__restrict__ Linv, int *__restrict__ status)
{
    __shared__ float S[NB * LDS_LD];    // L, column-major, S[c*LDS_LD + r]
    __shared__ float V[NB * LDS_LD];    // L^{-1}
    __shared__ float T[3 * 32 * TLD];   // scratch for the off-diagonal inverse blocks
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
        // 1. factor the diagonal 32 x 32 block in wave 0 (lanes 32..63 mirror 0..31)
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
                const float d = sqrtf(piv);
                const float inv = 1.0f / d;
                if (rr == c) a[c] = d;
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
        }
        __syncthreads();
        // 2. rows below: x L_JJ^T = a  (forward substitution along the row)
        const int nrow = NB - 32 - j0;
        if (tid < nrow) {
            const int i = j0 + 32 + tid;
            float x[32];
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                float v = S[(j0 + c) * LDS_LD + i];
#pragma unroll
                for (int k = 0; k < c; ++k) v = v - x[k] * S[(j0 + k) * LDS_LD + j0 + c];
                x[c] = v / S[(j0 + c) * LDS_LD + j0 + c];
            }
#pragma unroll
            for (int c = 0; c < 32; ++c) S[(j0 + c) * LDS_LD + i] = x[c];
        }
        __syncthreads();
        // 3. trailing update of rows/cols j0+32 .. 127 (lower 4 x 4 blocks)
        const int rem = NB - 32 - j0;
        const int nb4 = rem / 4;
        for (int b = tid; b < nb4 * nb4; b += 256) {
            const int bi = b % nb4, bk = b / nb4;
            if (bk > bi) continue;
            const int ib = j0 + 32 + 4 * bi, kb = j0 + 32 + 4 * bk;
            float acc[4][4];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = 0.0f;
            for (int c = 0; c < 32; ++c) {
                const float *col = S + (j0 + c) * LDS_LD;
                float xi[4], xk[4];
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    xi[x] = col[ib + x];
                    xk[x] = col[kb + x];
                }
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] += xi[x] * xk[y];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) S[(kb + y) * LDS_LD + ib + x] -= acc[x][y];
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

    // inverse, diagonal 32 x 32 blocks: wave w inverts block w; lane%32 = column
    {
        const int base = 32 * wave;
        const int jc = lane & 31;
        float x[32];
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            float v = (i == jc) ? 1.0f : 0.0f;
#pragma unroll
            for (int k = 0; k < i; ++k) v = v - S[(base + k) * LDS_LD + base + i] * x[k];
            x[i] = v / S[(base + i) * LDS_LD + base + i];
        }
        if (lane < 32) {
#pragma unroll
            for (int i = 0; i < 32; ++i) V[(base + jc) * LDS_LD + base + i] = x[i];
        }
    }
    __syncthreads();
    // off-diagonal blocks by distance d = I - J
    for (int d = 1; d < 4; ++d) {
        const int nblk = 4 - d;
        for (int e = tid; e < nblk * 1024; e += 256) {
            const int blk = e >> 10, rr = e & 31, cc = (e >> 5) & 31;
            const int J = blk, I = J + d;
            float v = 0.0f;
            for (int K = J; K < I; ++K)
                for (int q = 0; q < 32; ++q)
                    v += S[(32 * K + q) * LDS_LD + 32 * I + rr] * V[(32 * J + cc) * LDS_LD + 32 * K + q];
            T[blk * 32 * TLD + cc * TLD + rr] = v;
        }
        __syncthreads();
        for (int e = tid; e < nblk * 1024; e += 256) {
            const int blk = e >> 10, rr = e & 31, cc = (e >> 5) & 31;
            const int J = blk, I = J + d;
            float v = 0.0f;
            for (int q = 0; q < 32; ++q)
                v += V[(32 * I + q) * LDS_LD + 32 * I + rr] * T[blk * 32 * TLD + cc * TLD + q];
            V[(32 * J + cc) * LDS_LD + 32 * I + rr] = -v;
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
