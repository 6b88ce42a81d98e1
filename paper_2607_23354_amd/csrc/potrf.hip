// potrf.hip -- Cholesky factor and inverse of one 128 x 128 diagonal block.
//
// The blocked right-looking Cholesky (factor of Z, which is symmetric
// positive definite for distinct Euclidean points, Section 3.2) needs at each
// panel step the factor L11 of the diagonal block and, to turn the panel's
// triangular solve into an MFMA contraction, the explicit inverse L11^{-1}.
// Both are computed here by a single workgroup with the block held in LDS:
//
//   for each 32-column block J (right-looking):
//     1. one wave factors the 32 x 32 diagonal block and builds its inverse
//        in the same sweep, both as rank-1 updates on MFMA;
//     2. the blocks below are solved against it, L_IJ = A_IJ inv(L_JJ)^T,
//        and block row J of the inverse is scaled, Inv_JK = inv(L_JJ) Inv_JK;
//     3. the trailing blocks are updated, A_IK -= L_IJ L_KJ^T, and so are
//        the inverse's rows below, Inv_IK -= L_IJ Inv_JK; all but the block
//        the next factor needs run on waves 1..3 while wave 0 factors.
//   Steps 2 and 3 apply, block by block, L^{-1} = L_3^{-1} ... L_0^{-1}, where
//   L_J is the identity with block column J of L.
// Steps 2 and 3 are 32 x 32 x 32 products on MFMA
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

// Step-J products after the panel solve, as a list of independent 32 x 32 items:
//   trailing blocks    A_IK -= L_IJ L_KJ^T          (J < K <= I), pair (J+1, J+1) first
//   inverse rows I>J   Inv_IK -= L_IJ Inv_JK        (K <= J; Inv_IJ starts at 0)
// Items it = first, first + stride, ... < count run on this wave.
__device__ inline void step_products(float *S, float *V, int J, int first, int stride, int lane)
{
    const int j0 = 32 * J;
    const int rem = 3 - J;
    const int npair = rem * (rem + 1) / 2;
    const int nitems = npair + rem * (J + 1);
    for (int it = first; it < nitems; it += stride) {
        if (it < npair) {
            int Kr = 0;
            while ((Kr + 1) * (Kr + 2) / 2 <= it) ++Kr;
            const int Kc = it - Kr * (Kr + 1) / 2;
            const int I = J + 1 + Kr, K = J + 1 + Kc;
            v16f acc = blk_mma<true>(S + j0 * LDS_LD + 32 * I, LDS_LD, S + j0 * LDS_LD + 32 * K, LDS_LD,
                                     zero16(), lane);
            blk_store(S + (32 * K) * LDS_LD + 32 * I, LDS_LD, acc, lane, -1.0f, true);
        } else {
            const int u = it - npair;
            const int I = J + 1 + u / (J + 1), K = u % (J + 1);
            v16f acc = blk_mma<false>(S + j0 * LDS_LD + 32 * I, LDS_LD, V + (32 * K) * LDS_LD + j0, LDS_LD,
                                      zero16(), lane);
            blk_store(V + (32 * K) * LDS_LD + 32 * I, LDS_LD, acc, lane, -1.0f, K < J);
        }
    }
}

__device__ __forceinline__ void potrf128_body(float *__restrict__ A, int64_t ld, int64_t k0,
                                              float *__restrict__ Linv, int *__restrict__ status)
{
    __shared__ float S[NB * LDS_LD];    // L, column-major, S[c*LDS_LD + r]
    __shared__ float V[NB * LDS_LD];    // L^{-1}, same layout
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

    // columns c0 .. c0 + 31 of the factored block to A: L on and below the
    // diagonal, L^T above it (the mirror of an entry of an earlier, final column
    // or of the diagonal 32-block); threads t = 0 .. nt-1 of the caller
    auto write_cols = [&](int c0, int t, int nt) {
        for (int e = t; e < 32 * (NB / 4); e += nt) {
            const int c = c0 + (e >> 5), r4 = (e & 31) * 4;
            float4 v;
            v.x = (r4 + 0 >= c) ? S[c * LDS_LD + r4 + 0] : S[(r4 + 0) * LDS_LD + c];
            v.y = (r4 + 1 >= c) ? S[c * LDS_LD + r4 + 1] : S[(r4 + 1) * LDS_LD + c];
            v.z = (r4 + 2 >= c) ? S[c * LDS_LD + r4 + 2] : S[(r4 + 2) * LDS_LD + c];
            v.w = (r4 + 3 >= c) ? S[c * LDS_LD + r4 + 3] : S[(r4 + 3) * LDS_LD + c];
            *reinterpret_cast<float4 *>(Ablk + (int64_t)c * ld + r4) = v;
        }
    };

    // rows r0 .. r0 + 31 of the inverse to Linv (column-major, zero above the
    // diagonal)
    auto write_inv_rows = [&](int r0, int t, int nt) {
        for (int e = t; e < NB * 8; e += nt) {
            const int c = e >> 3, r4 = r0 + (e & 7) * 4;
            float4 w;
            w.x = (r4 + 0 >= c) ? V[c * LDS_LD + r4 + 0] : 0.0f;
            w.y = (r4 + 1 >= c) ? V[c * LDS_LD + r4 + 1] : 0.0f;
            w.z = (r4 + 2 >= c) ? V[c * LDS_LD + r4 + 2] : 0.0f;
            w.w = (r4 + 3 >= c) ? V[c * LDS_LD + r4 + 3] : 0.0f;
            *reinterpret_cast<float4 *>(Linv + c * NB + r4) = w;
        }
    };

    for (int J = 0; J < 4; ++J) {
        const int j0 = 32 * J;
        // 1. factor the diagonal 32 x 32 block in wave 0 and invert it in the same
        //    sweep, both as rank-1 updates on MFMA.  The symmetric block A is held
        //    whole in an accumulator: lane (h, b), register r holds A(a, b) with
        //    a = 8 (r / 4) + 4 h + r % 4, so row c (= column c) of A is register
        //    r_c of the lanes of half h_c.  Step c: l = A(:, c) / sqrt(A(c, c)) is
        //    column c of L; with m = l below the diagonal (zero elsewhere, and
        //    zero in the other half so the MFMA's k-slot h_c carries it),
        //    A -= m m^T.  The inverse Y (from I) takes the same elementary step
        //    L_c^{-1} as one update Y += g Y(c, :) with g_c = 1/sqrt(A(c, c)) - 1
        //    and g_k = -m_k / sqrt(A(c, c)) below.  Column c of L stays in the
        //    lanes that computed it (register r_c) until the sweep ends.
        if (wave != 0) {
            // block column J - 1 of L and block row J - 1 of the inverse are final
            // (step 2 of J - 1 was their last change): out to A and Linv now rather
            // than in the closing write-back; then the previous step's products that
            // this factor does not need (all but the trailing block (J, J), item 0),
            // on waves 1..3 beside the factor
            if (J > 0) {
                write_cols(32 * (J - 1), tid - 64, 192);
                write_inv_rows(32 * (J - 1), tid - 64, 192);
                step_products(S, V, J - 1, wave, 3, lane);
            }
        } else {
            const int b = lane & 31, h = lane >> 5;
            v16f accA, accY;
            float Lc[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int a = 8 * (r >> 2) + 4 * h + (r & 3);
                const int hiI = a > b ? a : b, loI = a > b ? b : a;
                accA[r] = S[(j0 + loI) * LDS_LD + j0 + hiI];  // lower triangle, mirrored
                accY[r] = (a == b) ? 1.0f : 0.0f;
                Lc[r] = 0.0f;
            }
            int firstbad = -1;  // branch-free pivot check keeps the sweep one basic block
            int bo = b, ho = h;
            // Columns in pairs (c, c + 1), both held by the same half (c even): column
            // c + 1 is brought up to date against column c on the VALU, so one wait on
            // the accumulator serves two pivots; then the four rank-1 MFMA updates.
#pragma unroll
            for (int c = 0; c < 32; c += 2) {
                const int r0 = 4 * (c >> 3) + (c & 3), r1 = r0 + 1, hc = (c >> 2) & 1;
                // lane predicates as 0/1 factors, recomputed per step (opaque lane ids
                // keep the compiler from precomputing every step's masks at once)
                asm volatile("" : "+v"(bo), "+v"(ho));
                const float fm = (ho == hc) ? 1.0f : 0.0f;
                const float fgt0 = (bo > c) ? fm : 0.0f, feq0 = (bo == c) ? fm : 0.0f;
                const float fgt1 = (bo > c + 1) ? fm : 0.0f, feq1 = (bo == c + 1) ? fm : 0.0f;
                // column c
                float piv0 = bcast(accA[r0], 32 * hc + c);
                const bool ok0 = (piv0 > 0.0f) && (piv0 < INFINITY);
                firstbad = (!ok0 && firstbad < 0) ? c : firstbad;
                piv0 = ok0 ? piv0 : 1.0f;
                const float inv0 = __builtin_amdgcn_rsqf(piv0);
                const float l0 = accA[r0] * inv0;       // L(b, c) in the lanes of half hc
                const float s = bcast(l0, 32 * hc + c + 1);  // L(c + 1, c)
                // column c + 1 after step c
                const float x1 = fmaf(-l0, s, accA[r1]);
                float piv1 = bcast(x1, 32 * hc + c + 1);
                const bool ok1 = (piv1 > 0.0f) && (piv1 < INFINITY);
                firstbad = (!ok1 && firstbad < 0) ? c + 1 : firstbad;
                piv1 = ok1 ? piv1 : 1.0f;
                const float inv1 = __builtin_amdgcn_rsqf(piv1);
                const float l1 = x1 * inv1;             // L(b, c + 1)
                Lc[r0] = fmaf(fm, l0 - Lc[r0], Lc[r0]);
                Lc[r1] = fmaf(fm, l1 - Lc[r1], Lc[r1]);
                const float m0 = fgt0 * l0, m1 = fgt1 * l1;
                // inverse: row c as it stands, row c + 1 after step c
                const float y0 = fm * accY[r0];
                const float y1 = fm * fmaf(-(s * inv0), accY[r0], accY[r1]);
                const float g0 = fmaf(feq0, inv0 - 1.0f, -(fgt0 * (l0 * inv0)));
                const float g1 = fmaf(feq1, inv1 - 1.0f, -(fgt1 * (l1 * inv1)));
                accA = __builtin_amdgcn_mfma_f32_32x32x2f32(-m0, m0, accA, 0, 0, 0);
                accA = __builtin_amdgcn_mfma_f32_32x32x2f32(-m1, m1, accA, 0, 0, 0);
                accY = __builtin_amdgcn_mfma_f32_32x32x2f32(g0, y0, accY, 0, 0, 0);
                accY = __builtin_amdgcn_mfma_f32_32x32x2f32(g1, y1, accY, 0, 0, 0);
            }
            if (firstbad >= 0 && lane == 0 && bad == 0) bad = (int)(k0 + j0 + firstbad + 1);
            // L(b, c) for the c of this half (entries above the diagonal land in the
            // upper triangle of S's diagonal block, which is never read), and the inverse
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int a = 8 * (r >> 2) + 4 * h + (r & 3);
                S[(j0 + a) * LDS_LD + j0 + b] = Lc[r];
                V[(j0 + b) * LDS_LD + j0 + a] = accY[r];
            }
        }
        __syncthreads();
        // 2. three independent 32 x 32 products, one per wave:
        //    blocks below:      L_IJ = A_IJ inv(L_JJ)^T            (I = J+1 .. 3)
        //    inverse, row J:    Inv_JK = inv(L_JJ) Inv_JK          (K = 0 .. J-1)
        //    (the block-level form of the same product of elementary inverses)
        if (wave < 3) {
            if (wave < 3 - J) {
                const int I = J + 1 + wave;
                v16f acc = blk_mma<true>(S + j0 * LDS_LD + 32 * I, LDS_LD, V + j0 * LDS_LD + j0, LDS_LD,
                                         zero16(), lane);
                blk_store(S + j0 * LDS_LD + 32 * I, LDS_LD, acc, lane, 1.0f, false);
            } else {
                const int K = wave - (3 - J);
                v16f acc = blk_mma<false>(V + j0 * LDS_LD + j0, LDS_LD, V + (32 * K) * LDS_LD + j0, LDS_LD,
                                          zero16(), lane);
                blk_store(V + (32 * K) * LDS_LD + j0, LDS_LD, acc, lane, 1.0f, false);
            }
        }
        __syncthreads();
        // 3. the trailing block (J+1, J+1), which the next factor needs first; the
        //    step's other products run beside that factor
        if (J < 3) {
            if (wave == 0) step_products(S, V, J, 0, 1 << 30, lane);
            __syncthreads();
        }
    }

    // the last block column of L and block row of the inverse (the others went
    // out during the steps)
    write_cols(96, tid, 256);
    write_inv_rows(96, tid, 256);
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
