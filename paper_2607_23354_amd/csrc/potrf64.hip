// potrf64.hip -- FP64 Cholesky factor and inverse of one 64 x 64 diagonal block.
//
// The FP64 blocked factor (the dense comparator's Cholesky of Z, Section 3.2)
// needs at each 64-column step the factor L11 of the diagonal block and its
// explicit inverse, which turns the panel's triangular solve into an MFMA
// contraction and is kept for the triangular solves of the substitution.
// One workgroup holds the block and the inverse in LDS:
//
//   for each 16-column block J (right-looking):
//     1. wave 0 factors the 16 x 16 diagonal block and inverts it in the same
//        sweep, both as rank-1 updates on the FP64 matrix cores;
//     2. the blocks below are solved against it, L_IJ = A_IJ inv(L_JJ)^T,
//        and block row J of the inverse is scaled, Inv_JK = inv(L_JJ) Inv_JK;
//     3. the trailing blocks are updated, A_IK -= L_IJ L_KJ^T, and so are
//        the inverse's rows below, Inv_IK -= L_IJ Inv_JK: wave 0 updates the
//        block (J+1, J+1) and goes straight on to its factor (step 1 of J+1)
//        while waves 1..3 update the rest.
//   Steps 2 and 3 apply, block by block, L^{-1} = L_3^{-1} ... L_0^{-1}, where
//   L_J is the identity with block column J of L; they are 16 x 16 x 16
//   products on v_mfma_f64_16x16x4 (one product per wave at a time).
//
// v_mfma_f64_16x16x4: lane l = 16 kq + q supplies A(q, kq) and B(kq, q) and
// holds D(kq + 4 v, q) in register v.
//
// A pivot that is not positive (or not finite) marks status[0] with the global
// pivot index + 1 and is replaced by 1 so the kernel still finishes.
#include "internal.hpp"

namespace mag {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int NB = 64;
constexpr int JB = 16;         // column block of the right-looking sweep
constexpr int LD = NB + 1;     // padded column stride of the LDS copies

__device__ inline double bcastd(double v, int src)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, src);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), src);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// 1/sqrt(p) for a normal p > 0: the hardware estimate and two Newton steps
// y <- y (3 - p y^2) / 2, each of which squares the relative error.
__device__ inline double rsqrt_nt(double p)
{
    double y = __builtin_amdgcn_rsq(p);
    const double hp = 0.5 * p;
    y = y * fma(-hp * y, y, 1.5);
    y = y * fma(-hp * y, y, 1.5);
    return y;
}

// D = X W for 16 x 16 blocks in column-major LDS: X(r, k) = X[k * xld + r],
// W(k, c) = W[c * wld + k] (WT: W(k, c) = W[k * wld + c]).
template <bool WT>
__device__ inline v4d blk16(const double *X, int xld, const double *W, int wld, int q, int kq)
{
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < JB; kk += 4) {
        const double a = X[(kk + kq) * xld + q];
        const double b = WT ? W[(kk + kq) * wld + q] : W[q * wld + kk + kq];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// dst(r, c) = [dst(r, c)] + sign acc(r, c) for a 16 x 16 block of column-major LDS
__device__ inline void blk16_store(double *dst, int ld, const v4d &acc, int q, int kq, double sign, bool accumulate)
{
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double *p = dst + q * ld + kq + 4 * v;
        *p = accumulate ? fma(sign, acc[v], *p) : sign * acc[v];
    }
}

__global__ void __launch_bounds__(256)
k_potrf64(double *__restrict__ A, int64_t ld, int64_t k0, double *__restrict__ Linv, int *__restrict__ status)
{
    __shared__ double S[NB * LD];   // A, then L: column-major S[c * LD + r], lower triangle
    __shared__ double V[NB * LD];   // L^{-1}, same layout
    __shared__ double Ys[JB * JB];  // inverse of the current 16 x 16 diagonal factor, Ys[c * JB + r]
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int q = lane & 15, kq = lane >> 4;
    double *Ablk = A + k0 * ld + k0;

    // the block: 8 loads of two entries per thread, all in flight before the
    // first LDS store (only the lower triangle is trusted)
    {
        double2 buf[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e2 = tid + 256 * i;
            const int c = e2 >> 5, r = (e2 & 31) * 2;
            buf[i] = *reinterpret_cast<const double2 *>(Ablk + (int64_t)c * ld + r);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e2 = tid + 256 * i;
            const int c = e2 >> 5, r = (e2 & 31) * 2;
            S[c * LD + r] = buf[i].x;
            S[c * LD + r + 1] = buf[i].y;
        }
    }
    if (tid == 0) bad = 0;
    __syncthreads();

    // Step J's products of stage 3 are items; item 0, the trailing block (J+1, J+1),
    // is the one the next factor needs, so wave 0 takes it and goes on to that
    // factor while waves 1..3 take the others.
    auto item = [&](int J, int it) {
        const int j0 = JB * J;
        const int rem = 3 - J;
        const int npair = rem * (rem + 1) / 2;
        if (it < npair) {
            int Kr = 0;
            while ((Kr + 1) * (Kr + 2) / 2 <= it) ++Kr;
            const int Kc = it - Kr * (Kr + 1) / 2;
            const int I = J + 1 + Kr, K = J + 1 + Kc;
            // A_IK -= L_IJ L_KJ^T, W(k, c) = L_KJ(c, k) = S[(j0 + k) LD + 16 K + c]
            const v4d d = blk16<true>(S + j0 * LD + JB * I, LD, S + j0 * LD + JB * K, LD, q, kq);
            blk16_store(S + (JB * K) * LD + JB * I, LD, d, q, kq, -1.0, true);
        } else {
            const int u = it - npair;
            const int I = J + 1 + u / (J + 1), K = u % (J + 1);
            // Inv_IK -= L_IJ Inv_JK; block (I, J) of the inverse is first written here (from zero)
            const v4d d = blk16<false>(S + j0 * LD + JB * I, LD, V + (JB * K) * LD + j0, LD, q, kq);
            blk16_store(V + (JB * K) * LD + JB * I, LD, d, q, kq, -1.0, K < J);
        }
    };
    auto nitems = [](int J) {
        const int rem = 3 - J;
        return rem * (rem + 1) / 2 + rem * (J + 1);
    };

    for (int J = 0; J < NB / JB; ++J) {
        const int j0 = JB * J;
        // 1. the diagonal block on wave 0 (after the trailing block it needs, from
        //    the previous step's products); the previous step's other products on
        //    waves 1..3.  The symmetric A_JJ is held whole in an
        //    accumulator (lane (q, kq), register v: A(kq + 4 v, q)), so row c of A
        //    (= column c) is register c / 4 of the lanes with kq = c % 4.  Step c:
        //    m = A(:, c) / sqrt(A(c, c)) below the diagonal (zero elsewhere and in
        //    the other lanes, so the MFMA's k-slot c % 4 carries it), A -= m m^T.
        //    The inverse Y (from I) takes the same elementary step: row c scaled
        //    by 1/sqrt(A(c, c)), then Y -= m Y(c, :).  Column c of L stays in the
        //    lanes that computed it (register c / 4) until the sweep ends.
        if (wave == 0) {
            if (J > 0) item(J - 1, 0);
            v4d a, y;
            double Lc[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = kq + 4 * v;
                const int hi = r > q ? r : q, lo = r > q ? q : r;
                a[v] = S[(j0 + lo) * LD + j0 + hi];
                y[v] = (r == q) ? 1.0 : 0.0;
                Lc[v] = 0.0;
            }
            int firstbad = -1;
#pragma unroll
            for (int c = 0; c < JB; ++c) {
                const int v = c >> 2, s = c & 3;
                double piv = bcastd(a[v], 16 * s + c);
                const bool ok = (piv > 0.0) && (piv < INFINITY);
                firstbad = (!ok && firstbad < 0) ? c : firstbad;
                piv = ok ? piv : 1.0;
                const double inv = rsqrt_nt(piv);
                const bool mine = kq == s;
                const double col = a[v] * inv;                 // A(q, c) / sqrt(piv) in lanes kq = s
                const double m = (mine && q > c) ? col : 0.0;
                Lc[v] = mine ? (q > c ? col : (q == c ? piv * inv : 0.0)) : Lc[v];
                y[v] = mine ? y[v] * inv : y[v];
                const double yr = mine ? y[v] : 0.0;
                a = __builtin_amdgcn_mfma_f64_16x16x4f64(-m, m, a, 0, 0, 0);
                y = __builtin_amdgcn_mfma_f64_16x16x4f64(-m, yr, y, 0, 0, 0);
            }
            // L(q, 4 v + kq) and Y(kq + 4 v, q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = 4 * v + kq;
                if (q >= c) S[(j0 + c) * LD + j0 + q] = Lc[v];
                Ys[q * JB + c] = y[v];
            }
            if (firstbad >= 0 && lane == 0 && bad == 0) bad = (int)(k0 + j0 + firstbad + 1);
        } else if (J > 0) {
            for (int it = wave; it < nitems(J - 1); it += 3) item(J - 1, it);
        }
        __syncthreads();
        // 2. three independent 16 x 16 products, one per wave, each in place on its
        //    own block:  L_IJ = A_IJ Y^T (I = J+1 .. 3),  Inv_JK = Y Inv_JK (K < J);
        //    wave 3 writes the inverse's diagonal block Y
        if (wave < 3) {
            if (wave < 3 - J) {
                const int I = J + 1 + wave;
                double *blk = S + j0 * LD + JB * I;
                const v4d d = blk16<true>(blk, LD, Ys, JB, q, kq);  // W(k, c) = Y(c, k) = Ys[k JB + c]
                blk16_store(blk, LD, d, q, kq, 1.0, false);
            } else {
                const int K = wave - (3 - J);
                double *blk = V + (JB * K) * LD + j0;
                const v4d d = blk16<false>(Ys, JB, blk, LD, q, kq);
                blk16_store(blk, LD, d, q, kq, 1.0, false);
            }
        } else {
            for (int e = lane; e < JB * JB; e += 64) {
                const int r = e & 15, c = e >> 4;
                V[(j0 + c) * LD + j0 + r] = Ys[c * JB + r];
            }
        }
        __syncthreads();
    }

    // L (lower triangle with the diagonal) and L^T above it; the inverse with zeros above
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int e2 = tid + 256 * i;
        const int c = e2 >> 5, r = (e2 & 31) * 2;
        double2 l, w;
        l.x = (r >= c) ? S[c * LD + r] : S[r * LD + c];
        l.y = (r + 1 >= c) ? S[c * LD + r + 1] : S[(r + 1) * LD + c];
        w.x = (r >= c) ? V[c * LD + r] : 0.0;
        w.y = (r + 1 >= c) ? V[c * LD + r + 1] : 0.0;
        *reinterpret_cast<double2 *>(Ablk + (int64_t)c * ld + r) = l;
        *reinterpret_cast<double2 *>(Linv + c * NB + r) = w;
    }
    if (tid == 0 && bad != 0) atomicCAS(&status[kStBreakdown], 0, bad);
}

}  // namespace

void launch_potrf64(hipStream_t s, double *A, int64_t ld, int64_t k0, double *Linv, int *status)
{
    hipLaunchKernelGGL(k_potrf64, dim3(1), dim3(256), 0, s, A, ld, k0, Linv, status);
}

}  // namespace mag
