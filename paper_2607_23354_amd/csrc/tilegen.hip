// tilegen.hip -- the tile generator: blocks of Z = exp[-t d] formed on the fly
// from coordinates staged in LDS, with exact coordinate differences
// d_jk = sqrt(sum_l (x_jl - x_kl)^2) (never the |x|^2 + |y|^2 - 2 x.y form).
//
// Section 2 of the paper defines Z = exp[-t d] with Euclidean d; this file
// only evaluates it.  The squared distance is accumulated over l in ascending
// order with every product and sum rounded separately (no contraction), which
// is the order the oracle uses, so both sides see the same d_jk bits.
#include "internal.hpp"

#include <cmath>

namespace mag {
namespace {

constexpr int kRows = 128;   // rows of Z per workgroup block
constexpr int kCols = 64;    // columns of Z per workgroup block
constexpr int kLC = 8;       // coordinates staged per LDS pass
constexpr int kThreads = 256;
constexpr int kPerThread = kRows * kCols / kThreads;  // 32 entries

// Map a linear block index onto the lower block set {(I, Jc) : Jc <= 2I+1},
// where I counts 128-row tiles and Jc counts 64-column blocks.  Row tile I
// owns blocks [I(I+1), (I+1)(I+2)).
__device__ inline void lower_block(int64_t idx, int64_t &I, int64_t &Jc)
{
    int64_t r = (int64_t)((sqrt(4.0 * (double)idx + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) > idx) --r;
    while ((r + 1) * (r + 2) <= idx) ++r;
    I = r;
    Jc = idx - r * (r + 1);
}

__device__ inline double sq_acc(double s, double e)
{
#pragma clang fp contract(off)
    double p = e * e;
    return s + p;
}

// Stage coordinates [l0, l0+lc) of `count` consecutive points starting at
// `first` into S[l][count] (zero beyond n).
__device__ inline void stage(double *S, int count, const double *X, int64_t n, int m,
                             int64_t first, int l0, int lc)
{
    for (int e = threadIdx.x; e < lc * count; e += blockDim.x) {
        int l = e / count, p = e % count;
        int64_t j = first + p;
        S[l * count + p] = (j < n) ? X[j * m + l0 + l] : 0.0;
    }
}

// Squared distances of the 32 entries (row r, columns c0 + 2*c ... ) of a
// 128 x 64 block.  Thread layout: r = tid & 127, column parity h = tid >> 7,
// entry c covers column 2c + h, so a fixed c is written by 128 consecutive rows.
__device__ inline void block_sqdist(double (&s)[kPerThread], const double *X, int64_t n, int m,
                                    int64_t row0, int64_t col0, double *Sr, double *Sc)
{
    const int r = threadIdx.x & (kRows - 1);
    const int h = threadIdx.x >> 7;
#pragma unroll
    for (int c = 0; c < kPerThread; ++c) s[c] = 0.0;
    for (int l0 = 0; l0 < m; l0 += kLC) {
        int lc = min(kLC, m - l0);
        __syncthreads();
        stage(Sr, kRows, X, n, m, row0, l0, lc);
        stage(Sc, kCols, X, n, m, col0, l0, lc);
        __syncthreads();
        for (int l = 0; l < lc; ++l) {
            double xr = Sr[l * kRows + r];
#pragma unroll
            for (int c = 0; c < kPerThread; ++c) {
                double e = xr - Sc[l * kCols + 2 * c + h];
                s[c] = sq_acc(s[c], e);
            }
        }
    }
}

template <int KERN = kKernExp>
__device__ __forceinline__ void tilegen32_body(const double *__restrict__ X, int64_t n, int m,
                                               double t, float *__restrict__ A, int64_t npad,
                                               float shift, int64_t blk, int *__restrict__ status)
{
    __shared__ double Sr[kLC * kRows];
    __shared__ double Sc[kLC * kCols];
    int64_t I, Jc;
    lower_block(blk, I, Jc);
    const int64_t row0 = I * kRows, col0 = Jc * kCols;
    double s[kPerThread];
    block_sqdist(s, X, n, m, row0, col0, Sr, Sc);
    const int r = threadIdx.x & (kRows - 1);
    const int h = threadIdx.x >> 7;
    const int64_t j = row0 + r;
    const float tf = (float)t;
#pragma unroll
    for (int c = 0; c < kPerThread; ++c) {
        const int64_t k = col0 + 2 * c + h;
        float v;
        if (j == k)
            v = ((KERN == kKernShiftDist) ? tf : 1.0f) + shift;
        else if (j >= n || k >= n)
            v = 0.0f;
        else {
            if (status && s[c] == 0.0) status[kStDuplicate] = 1;  // Z singular
            if (KERN == kKernShiftDist)
                v = (float)(t - sqrt(s[c]));  // c - d_jk, formed in FP64
            else
                v = expf(-(tf * sqrtf((float)s[c])));
        }
        A[k * npad + j] = v;
    }
}

template <int KERN>
__global__ void __launch_bounds__(kThreads)
k_tilegen32(const double *__restrict__ X, int64_t n, int m, double t, float *__restrict__ A,
            int64_t npad, float shift, int *__restrict__ status)
{
    tilegen32_body<KERN>(X, n, m, t, A, npad, shift, blockIdx.x, status);
}

// Batched: one launch for every active problem of a batch.
__global__ void __launch_bounds__(kThreads)
k_tilegen32_b(const BProb *__restrict__ P, BWork w)
{
    const int i = bfind(w.pref, w.na, blockIdx.x);
    const BProb &q = P[w.plist[i]];
    if (!q.active) return;
    tilegen32_body(q.X, q.n, q.m, q.t, q.A, q.npad, (float)q.shift, blockIdx.x - w.pref[i], nullptr);
}

__global__ void __launch_bounds__(kThreads)
k_tilegen64(const double *__restrict__ X, int64_t n, int m, double t, double *__restrict__ A)
{
    __shared__ double Sr[kLC * kRows];
    __shared__ double Sc[kLC * kCols];
    int64_t I, Jc;
    lower_block(blockIdx.x, I, Jc);
    const int64_t row0 = I * kRows, col0 = Jc * kCols;
    if (col0 >= n) return;  // whole block beyond the matrix (uniform per block)
    double s[kPerThread];
    block_sqdist(s, X, n, m, row0, col0, Sr, Sc);
    const int r = threadIdx.x & (kRows - 1);
    const int h = threadIdx.x >> 7;
    const int64_t j = row0 + r;
    if (j >= n) return;
#pragma unroll
    for (int c = 0; c < kPerThread; ++c) {
        const int64_t k = col0 + 2 * c + h;
        if (k > j || k >= n) continue;
        double v = (j == k) ? 1.0 : exp(-(t * sqrt(s[c])));
        A[k * n + j] = v;
    }
}

// FP64 Z into the padded layout of the FP32 factor (npad x npad column-major,
// lower triangle and the 128 x 128 diagonal tiles, identity padding), for the
// FP64 blocked factor; the entries are those of k_tilegen64.
__global__ void __launch_bounds__(kThreads)
k_tilegen64p(const double *__restrict__ X, int64_t n, int m, double t, double *__restrict__ A, int64_t npad,
             int *__restrict__ status)
{
    __shared__ double Sr[kLC * kRows];
    __shared__ double Sc[kLC * kCols];
    int64_t I, Jc;
    lower_block(blockIdx.x, I, Jc);
    const int64_t row0 = I * kRows, col0 = Jc * kCols;
    double s[kPerThread];
    block_sqdist(s, X, n, m, row0, col0, Sr, Sc);
    const int r = threadIdx.x & (kRows - 1);
    const int h = threadIdx.x >> 7;
    const int64_t j = row0 + r;
#pragma unroll
    for (int c = 0; c < kPerThread; ++c) {
        const int64_t k = col0 + 2 * c + h;
        double v;
        if (j == k)
            v = 1.0;
        else if (j >= n || k >= n)
            v = 0.0;
        else {
            if (status && s[c] == 0.0) status[kStDuplicate] = 1;  // Z singular
            v = exp(-(t * sqrt(s[c])));
        }
        A[k * npad + j] = v;
    }
}

// Per-block minimum of d_jk^2 over j > k inside the block.
__global__ void __launch_bounds__(kThreads)
k_dmin2_partial(const double *__restrict__ X, int64_t n, int m, double *__restrict__ partial)
{
    __shared__ double Sr[kLC * kRows];
    __shared__ double Sc[kLC * kCols];
    __shared__ double red[kThreads];
    int64_t I, Jc;
    lower_block(blockIdx.x, I, Jc);
    const int64_t row0 = I * kRows, col0 = Jc * kCols;
    double best = INFINITY;
    if (col0 < n) {  // uniform per block
        double s[kPerThread];
        block_sqdist(s, X, n, m, row0, col0, Sr, Sc);
        const int r = threadIdx.x & (kRows - 1);
        const int h = threadIdx.x >> 7;
        const int64_t j = row0 + r;
#pragma unroll
        for (int c = 0; c < kPerThread; ++c) {
            const int64_t k = col0 + 2 * c + h;
            if (j < n && k < j) best = fmin(best, s[c]);
        }
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256)
k_min_reduce(const double *__restrict__ partial, int64_t np, double *__restrict__ out)
{
    __shared__ double red[256];
    double best = INFINITY;
    for (int64_t i = threadIdx.x; i < np; i += 256) best = fmin(best, partial[i]);
    red[threadIdx.x] = best;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_check_finite(const double *__restrict__ X, int64_t count, int *status)
{
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(X[i]);
    if (bad) status[kStNonFinite] = 1;
}

int64_t lower_blocks(int64_t rows)
{
    int64_t T = (rows + kRows - 1) / kRows;
    return T * (T + 1);
}

}  // namespace

void launch_tilegen32(hipStream_t s, const double *X, int64_t n, int m, double t, float *A,
                      int64_t npad, float shift, int *status, int kernel)
{
    if (kernel == kKernShiftDist)
        hipLaunchKernelGGL(k_tilegen32<kKernShiftDist>, dim3((unsigned)lower_blocks(npad)), dim3(kThreads), 0, s, X,
                           n, m, t, A, npad, shift, status);
    else
        hipLaunchKernelGGL(k_tilegen32<kKernExp>, dim3((unsigned)lower_blocks(npad)), dim3(kThreads), 0, s, X, n,
                           m, t, A, npad, shift, status);
}

void launch_tilegen64(hipStream_t s, const double *X, int64_t n, int m, double t, double *A)
{
    hipLaunchKernelGGL(k_tilegen64, dim3((unsigned)lower_blocks(n)), dim3(kThreads), 0, s, X, n, m,
                       t, A);
}

void launch_tilegen64p(hipStream_t s, const double *X, int64_t n, int m, double t, double *A, int64_t npad,
                       int *status)
{
    hipLaunchKernelGGL(k_tilegen64p, dim3((unsigned)lower_blocks(npad)), dim3(kThreads), 0, s, X, n, m, t, A, npad,
                       status);
}

void launch_dmin2(hipStream_t s, const double *X, int64_t n, int m, double *partial, int64_t *np,
                  double *out_min2)
{
    int64_t nb = lower_blocks(n);
    hipLaunchKernelGGL(k_dmin2_partial, dim3((unsigned)nb), dim3(kThreads), 0, s, X, n, m, partial);
    hipLaunchKernelGGL(k_min_reduce, dim3(1), dim3(256), 0, s, partial, nb, out_min2);
    if (np) *np = nb;
}

void launch_check_finite(hipStream_t s, const double *X, int64_t count, int *status)
{
    int64_t blocks = (count + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, s, X, count, status);
}

size_t dmin_partial_doubles(int64_t n) { return (size_t)lower_blocks(n); }

int64_t tilegen32_blocks(int64_t npad) { return lower_blocks(npad); }

void launch_tilegen32_b(hipStream_t s, const BProb *P, const BWork &w)
{
    if (w.total > 0)
        hipLaunchKernelGGL(k_tilegen32_b, dim3((unsigned)w.total), dim3(kThreads), 0, s, P, w);
}

}  // namespace mag
