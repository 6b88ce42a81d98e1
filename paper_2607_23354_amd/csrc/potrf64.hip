// potrf64.hip -- FP64 Cholesky factor and inverse of one 64 x 64 diagonal block.
//
// The FP64 blocked factor (the dense comparator's Cholesky of Z, Section 3.2)
// needs at each 64-column step the factor L11 of the diagonal block and its
// explicit inverse, which turns the panel's triangular solve into an MFMA
// contraction and is kept for the triangular solves of the substitution.
// One workgroup holds the block and the inverse in LDS:
//
//   for each 16-column block J (right-looking):
//     1. wave 0 factors the 16 x 16 diagonal block and inverts it (lane r
//        holds row r of both; column c of L and row c of the inverse are
//        broadcast from lane c);
//     2. the blocks below are solved against it, L_IJ = A_IJ inv(L_JJ)^T,
//        and block row J of the inverse is scaled, Inv_JK = inv(L_JJ) Inv_JK;
//     3. the trailing lower triangle is updated, A_IK -= L_IJ L_KJ^T, and so
//        are the inverse's rows below, Inv_IK -= L_IJ Inv_JK.
//   Steps 2 and 3 apply, block by block, L^{-1} = L_3^{-1} ... L_0^{-1}, where
//   L_J is the identity with block column J of L.
//
// A pivot that is not positive (or not finite) marks status[0] with the global
// pivot index + 1 and is replaced by 1 so the kernel still finishes.
#include "internal.hpp"

namespace mag {
namespace {

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

__global__ void __launch_bounds__(256)
k_potrf64(double *__restrict__ A, int64_t ld, int64_t k0, double *__restrict__ Linv, int *__restrict__ status)
{
    __shared__ double S[NB * LD];   // A, then L: column-major S[c * LD + r], lower triangle
    __shared__ double V[NB * LD];   // L^{-1}, same layout, lower triangle
    __shared__ double Y[JB * JB];   // inverse of the current 16 x 16 diagonal factor, Y[c * JB + r]
    __shared__ int bad;
    const int tid = threadIdx.x;
    double *Ablk = A + k0 * ld + k0;

    // lower triangle (the upper half of the block may be stale)
    for (int e = tid; e < NB * NB; e += 256) {
        const int c = e >> 6, r = e & 63;
        if (r >= c) S[c * LD + r] = Ablk[(int64_t)c * ld + r];
        V[c * LD + r] = 0.0;
    }
    if (tid == 0) bad = 0;
    __syncthreads();

    for (int J = 0; J < NB / JB; ++J) {
        const int j0 = JB * J;
        // 1. the diagonal block: lane r < 16 holds row r of A_JJ (a) and of its
        //    inverse (y), and builds row r of L_JJ (l)
        if (tid < 64) {
            const int r = tid;
            double a[JB], y[JB], l[JB];
#pragma unroll
            for (int c = 0; c < JB; ++c) {
                const int hi = r > c ? r : c, lo = r > c ? c : r;
                a[c] = (r < JB) ? S[(j0 + lo) * LD + j0 + hi] : 0.0;
                y[c] = (r == c) ? 1.0 : 0.0;
                l[c] = 0.0;
            }
            int firstbad = -1;
#pragma unroll
            for (int c = 0; c < JB; ++c) {
                double piv = bcastd(a[c], c);
                const bool ok = (piv > 0.0) && (piv < INFINITY);
                firstbad = (!ok && firstbad < 0) ? c : firstbad;
                piv = ok ? piv : 1.0;
                const double d = sqrt(piv), inv = 1.0 / d;
                // column c of L: l_r = a_rc / d below the diagonal, d on it
                const double lr = (r > c) ? a[c] * inv : (r == c ? d : 0.0);
                l[c] = lr;
                // row c of the inverse: Y(c, :) / d, then Y(r, :) -= L(r, c) Y(c, :)
                if (r == c) {
#pragma unroll
                    for (int k = 0; k <= c; ++k) y[k] *= inv;
                }
#pragma unroll
                for (int k = 0; k <= c; ++k) {
                    const double yc = bcastd(y[k], c);
                    if (r > c) y[k] = fma(-lr, yc, y[k]);
                }
                // trailing entries of the block: a_rj -= l_r l_j (j > c)
#pragma unroll
                for (int j = c + 1; j < JB; ++j) {
                    const double lj = bcastd(lr, j);
                    a[j] = fma(-lr, lj, a[j]);
                }
            }
            if (r < JB) {
#pragma unroll
                for (int c = 0; c < JB; ++c) {
                    if (r >= c) S[(j0 + c) * LD + j0 + r] = l[c];
                    Y[c * JB + r] = y[c];
                }
            }
            if (firstbad >= 0 && r == 0 && bad == 0) bad = (int)(k0 + j0 + firstbad + 1);
        }
        __syncthreads();
        // 2. blocks below, L_IJ = A_IJ Y^T (rows j0 + 16 .. 63), and block row J of
        //    the inverse, Inv_JK = Y Inv_JK (columns 0 .. j0 - 1): 768 entries, each
        //    a 16-term product, computed before any is stored
        {
            const int nbelow = (NB - j0 - JB) * JB;
            double res[3];
            int idx[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int e = tid + 256 * u;
                double s = 0.0;
                idx[u] = -1;
                if (e < nbelow) {
                    const int rr = j0 + JB + e % (NB - j0 - JB), c = e / (NB - j0 - JB);
#pragma unroll
                    for (int k = 0; k < JB; ++k) s = fma(S[(j0 + k) * LD + rr], Y[k * JB + c], s);
                    idx[u] = (j0 + c) * LD + rr;
                } else if (e < nbelow + JB * j0) {
                    const int f = e - nbelow;
                    const int rr = f % JB, c = f / JB;
                    for (int k = 0; k <= rr; ++k) s = fma(Y[k * JB + rr], V[c * LD + j0 + k], s);
                    idx[u] = NB * LD + c * LD + j0 + rr;  // marks V
                }
                res[u] = s;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                if (idx[u] >= NB * LD) V[idx[u] - NB * LD] = res[u];
                else if (idx[u] >= 0) S[idx[u]] = res[u];
            }
            // the diagonal block of the inverse
            if (tid < JB * JB) {
                const int rr = tid % JB, c = tid / JB;
                V[(j0 + c) * LD + j0 + rr] = (rr >= c) ? Y[c * JB + rr] : 0.0;
            }
        }
        __syncthreads();
        // 3. trailing lower triangle and the inverse's rows below block J
        if (J + 1 < NB / JB) {
            const int base = j0 + JB, w = NB - base;
            const int ntri = w * w;  // square index space, lower half used
            for (int e = tid; e < ntri; e += 256) {
                const int rr = base + e % w, c = base + e / w;
                if (rr < c) continue;
                double s = S[c * LD + rr];
#pragma unroll
                for (int k = 0; k < JB; ++k) s = fma(-S[(j0 + k) * LD + rr], S[(j0 + k) * LD + c], s);
                S[c * LD + rr] = s;
            }
            const int ninv = w * (j0 + JB);
            for (int e = tid; e < ninv; e += 256) {
                const int rr = base + e % w, c = e / w;
                double s = V[c * LD + rr];
#pragma unroll
                for (int k = 0; k < JB; ++k) s = fma(-S[(j0 + k) * LD + rr], V[c * LD + j0 + k], s);
                V[c * LD + rr] = s;
            }
        }
        __syncthreads();
    }

    // L (lower triangle with the diagonal) and L^T above it; the inverse with zeros above
    for (int e = tid; e < NB * NB; e += 256) {
        const int c = e >> 6, r = e & 63;
        Ablk[(int64_t)c * ld + r] = (r >= c) ? S[c * LD + r] : S[r * LD + c];
        Linv[c * NB + r] = (r >= c) ? V[c * LD + r] : 0.0;
    }
    if (tid == 0 && bad != 0) atomicCAS(&status[kStBreakdown], 0, bad);
}

}  // namespace

void launch_potrf64(hipStream_t s, double *A, int64_t ld, int64_t k0, double *Linv, int *status)
{
    hipLaunchKernelGGL(k_potrf64, dim3(1), dim3(256), 0, s, A, ld, k0, Linv, status);
}

}  // namespace mag
