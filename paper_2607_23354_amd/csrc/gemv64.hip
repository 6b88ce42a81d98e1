// gemv64.hip -- FP64 matrix-free product y = Z v with Z = exp[-t d]
// regenerated tile by tile from the coordinates (Section 2), used for the
// refinement residual r = 1 - Z w and for the Krylov matvecs.  Nothing of Z is
// stored: the cost is n^2 FP64 distance + exp evaluations, the traffic only
// O(n m).  The entry is formed exactly as the tile generator forms it
// (exact differences, uncontracted squared sum in ascending l, sqrt, then
// exp(-(t d))), in FP64.
//
// Grid: (row blocks of 256 rows, one row per thread) x (column splits).  Each
// workgroup stages 256-column chunks of coordinates and v in LDS and sweeps
// its column range; partial row sums go to a split-major buffer and a second
// kernel adds the splits in fixed order (deterministic), optionally forming
// b - Z v and its max-norm.
#include "internal.hpp"

#include <cmath>

namespace mag {
namespace {

constexpr int RT = 256;   // rows per block (threads)
constexpr int CH = 256;   // columns per LDS chunk
constexpr int MMAX_LDS = 8;   // compile-time dimensions up to 8 stage coordinates in LDS

__device__ inline double sq_acc(double s, double e)
{
#pragma clang fp contract(off)
    double p = e * e;
    return s + p;
}

template <int M>
__global__ void __launch_bounds__(RT)
k_zmv_partial(const double *__restrict__ X, int64_t n, int m_rt, double t,
              const double *__restrict__ v, double *__restrict__ partial, int64_t cps,
              int64_t npad)
{
    __shared__ double Xc[MMAX_LDS * CH];
    __shared__ double vc[CH];
    const int m = (M > 0) ? M : m_rt;
    const int64_t j = (int64_t)blockIdx.x * RT + threadIdx.x;
    const int64_t c_lo = (int64_t)blockIdx.y * cps;
    const int64_t c_hi = min(n, c_lo + cps);
    const bool live = j < n;
    double acc = 0.0;

    if (M > 0) {
        double xr[M > 0 ? M : 1];
#pragma unroll
        for (int l = 0; l < (M > 0 ? M : 1); ++l) xr[l] = live ? X[j * M + l] : 0.0;
        for (int64_t k0 = c_lo; k0 < c_hi; k0 += CH) {
            const int cnt = (int)min((int64_t)CH, c_hi - k0);
            __syncthreads();
            for (int e = threadIdx.x; e < cnt * M; e += RT) {
                const int p = e / M, l = e % M;
                Xc[l * CH + p] = X[(k0 + p) * M + l];
            }
            if (threadIdx.x < cnt) vc[threadIdx.x] = v[k0 + threadIdx.x];
            __syncthreads();
            if (live) {
                for (int c = 0; c < cnt; ++c) {
                    double s = 0.0;
#pragma unroll
                    for (int l = 0; l < M; ++l) s = sq_acc(s, xr[l] - Xc[l * CH + c]);
                    const double z = (k0 + c == j) ? 1.0 : exp(-(t * sqrt(s)));
                    acc = fma(z, vc[c], acc);
                }
            }
        }
    } else {
        // runtime m: coordinates read directly (L1/L2 cached); v staged per chunk
        for (int64_t k0 = c_lo; k0 < c_hi; k0 += CH) {
            const int cnt = (int)min((int64_t)CH, c_hi - k0);
            __syncthreads();
            if (threadIdx.x < cnt) vc[threadIdx.x] = v[k0 + threadIdx.x];
            __syncthreads();
            if (live) {
                const double *xj = X + j * m;
                for (int c = 0; c < cnt; ++c) {
                    const double *xk = X + (k0 + c) * m;
                    double s = 0.0;
                    for (int l = 0; l < m; ++l) s = sq_acc(s, xj[l] - xk[l]);
                    const double z = (k0 + c == j) ? 1.0 : exp(-(t * sqrt(s)));
                    acc = fma(z, vc[c], acc);
                }
            }
        }
    }
    if (j < npad) partial[(int64_t)blockIdx.y * npad + j] = live ? acc : 0.0;
}

// mode 0: y = sum_s partial;  mode 1: y = b - sum_s partial (b == NULL: ones),
// and per-block max |y| into blkmax.
__global__ void __launch_bounds__(256)
k_zmv_reduce(const double *__restrict__ partial, int64_t npad, int64_t n, int splits,
             double *__restrict__ y, const double *__restrict__ b, int mode,
             double *__restrict__ blkmax)
{
    __shared__ double red[256];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double val = 0.0;
    if (j < npad) {
        double s = 0.0;
        for (int q = 0; q < splits; ++q) s += partial[(int64_t)q * npad + j];
        if (j >= n) val = 0.0;
        else if (mode == 0) val = s;
        else val = (b ? b[j] : 1.0) - s;
        y[j] = val;
    }
    if (mode == 1) {
        red[threadIdx.x] = fabs(val);
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0) blkmax[blockIdx.x] = red[0];
    }
}

__global__ void __launch_bounds__(256) k_max_final(const double *blkmax, int64_t nb, double *out)
{
    __shared__ double red[256];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += 256) v = fmax(v, blkmax[i]);
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

struct Plan {
    int64_t rowblocks, splits, cps, npad;
};

Plan plan_for(int64_t n)
{
    Plan p;
    p.npad = round_up(n, kPad);
    p.rowblocks = (n + RT - 1) / RT;
    int64_t s = (2048 + p.rowblocks - 1) / p.rowblocks;
    int64_t maxs = (n + CH - 1) / CH;
    if (s > maxs) s = maxs;
    if (s > 64) s = 64;
    if (s < 1) s = 1;
    p.cps = round_up((n + s - 1) / s, CH);
    p.splits = (n + p.cps - 1) / p.cps;
    return p;
}

}  // namespace

size_t zmv_partial_doubles(int64_t n)
{
    Plan p = plan_for(n);
    return (size_t)(p.splits * p.npad + p.npad / 256 + 8);
}

void launch_zmv(hipStream_t s, const double *X, int64_t n, int m, double t, const double *v,
                double *y, const double *b, int mode, double *partial, double *out_norm)
{
    Plan p = plan_for(n);
    dim3 grid((unsigned)p.rowblocks, (unsigned)p.splits);
    switch (m) {
    case 1: hipLaunchKernelGGL(k_zmv_partial<1>, grid, dim3(RT), 0, s, X, n, m, t, v, partial, p.cps, p.npad); break;
    case 2: hipLaunchKernelGGL(k_zmv_partial<2>, grid, dim3(RT), 0, s, X, n, m, t, v, partial, p.cps, p.npad); break;
    case 3: hipLaunchKernelGGL(k_zmv_partial<3>, grid, dim3(RT), 0, s, X, n, m, t, v, partial, p.cps, p.npad); break;
    case 4: hipLaunchKernelGGL(k_zmv_partial<4>, grid, dim3(RT), 0, s, X, n, m, t, v, partial, p.cps, p.npad); break;
    case 5: hipLaunchKernelGGL(k_zmv_partial<5>, grid, dim3(RT), 0, s, X, n, m, t, v, partial, p.cps, p.npad); break;
    case 6: hipLaunchKernelGGL(k_zmv_partial<6>, grid, dim3(RT), 0, s, X, n, m, t, v, partial, p.cps, p.npad); break;
    case 7: hipLaunchKernelGGL(k_zmv_partial<7>, grid, dim3(RT), 0, s, X, n, m, t, v, partial, p.cps, p.npad); break;
    case 8: hipLaunchKernelGGL(k_zmv_partial<8>, grid, dim3(RT), 0, s, X, n, m, t, v, partial, p.cps, p.npad); break;
    default: hipLaunchKernelGGL(k_zmv_partial<0>, grid, dim3(RT), 0, s, X, n, m, t, v, partial, p.cps, p.npad); break;
    }
    // rows beyond rowblocks*RT but below npad are written by the reduce kernel as zero
    const int64_t rb = p.npad / 256;
    double *blkmax = partial + p.splits * p.npad;
    // the partial kernel covers rows < rowblocks*RT; make rows up to npad defined
    hipLaunchKernelGGL(k_zmv_reduce, dim3((unsigned)rb), dim3(256), 0, s, partial, p.npad, n,
                       (int)p.splits, y, b, mode, blkmax);
    if (mode == 1 && out_norm)
        hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, blkmax, rb, out_norm);
}

}  // namespace mag
