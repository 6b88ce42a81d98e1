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
__device__ __forceinline__ void zmv_partial_body(const double *__restrict__ X, int64_t n, int m_rt,
                                                 double t, const double *__restrict__ v,
                                                 double *__restrict__ partial, int64_t cps,
                                                 int64_t npad, int64_t bx, int64_t by)
{
    __shared__ double Xc[MMAX_LDS * CH];
    __shared__ double vc[CH];
    const int m = (M > 0) ? M : m_rt;
    const int64_t j = bx * RT + threadIdx.x;
    const int64_t c_lo = by * cps;
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
    if (j < npad) partial[by * npad + j] = live ? acc : 0.0;
}

template <int M>
__global__ void __launch_bounds__(RT)
k_zmv_partial(const double *__restrict__ X, int64_t n, int m_rt, double t,
              const double *__restrict__ v, double *__restrict__ partial, int64_t cps,
              int64_t npad)
{
    zmv_partial_body<M>(X, n, m_rt, t, v, partial, cps, npad, blockIdx.x, blockIdx.y);
}

// mode 0: y = sum_s partial;  mode 1: y = b - sum_s partial (b == NULL: ones),
// and per-block max |y| into blkmax.
__device__ __forceinline__ void zmv_reduce_body(const double *__restrict__ partial, int64_t npad,
                                                int64_t n, int splits, double *__restrict__ y,
                                                const double *__restrict__ b, int mode,
                                                double *__restrict__ blkmax, int64_t bx)
{
    __shared__ double red[256];
    const int64_t j = bx * 256 + threadIdx.x;
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
        if (threadIdx.x == 0) blkmax[bx] = red[0];
    }
}

__global__ void __launch_bounds__(256)
k_zmv_reduce(const double *__restrict__ partial, int64_t npad, int64_t n, int splits,
             double *__restrict__ y, const double *__restrict__ b, int mode,
             double *__restrict__ blkmax)
{
    zmv_reduce_body(partial, npad, n, splits, y, b, mode, blkmax, blockIdx.x);
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

__host__ __device__ inline Plan plan_for(int64_t n)
{
    Plan p;
    p.npad = (n + kPad - 1) / kPad * kPad;
    p.rowblocks = (n + RT - 1) / RT;
    int64_t s = (2048 + p.rowblocks - 1) / p.rowblocks;
    int64_t maxs = (n + CH - 1) / CH;
    if (s > maxs) s = maxs;
    if (s > 64) s = 64;
    if (s < 1) s = 1;
    p.cps = ((n + s - 1) / s + CH - 1) / CH * CH;
    p.splits = (n + p.cps - 1) / p.cps;
    return p;
}

// Batched Z v: work units of problem p = rowblocks * splits (row block major).
template <int M>
__global__ void __launch_bounds__(RT)
k_zmv_partial_b(const BProb *__restrict__ P, BWork w, int v_slot)
{
    const int i = bfind(w.pref, w.na, blockIdx.x);
    const BProb &q = P[w.plist[i]];
    if (!q.active) return;
    const Plan pl = plan_for(q.n);
    const int64_t u = blockIdx.x - w.pref[i];
    zmv_partial_body<M>(q.X, q.n, q.m, q.t, q.vec + (int64_t)v_slot * q.npad, q.partial, pl.cps,
                        q.npad, u / pl.splits, u % pl.splits);
}

// Batched reduce (units = npad/256 per problem); mode 1 writes b - Z v with b
// from b_slot (b_slot < 0: ones) and per-block maxima after the split partials.
__global__ void __launch_bounds__(256)
k_zmv_reduce_b(const BProb *__restrict__ P, BWork w, int y_slot, int b_slot, int mode)
{
    const int i = bfind(w.pref, w.na, blockIdx.x);
    const BProb &q = P[w.plist[i]];
    if (!q.active) return;
    const Plan pl = plan_for(q.n);
    const int64_t u = blockIdx.x - w.pref[i];
    zmv_reduce_body(q.partial, q.npad, q.n, (int)pl.splits, q.vec + (int64_t)y_slot * q.npad,
                    b_slot >= 0 ? q.vec + (int64_t)b_slot * q.npad : nullptr, mode,
                    q.partial + pl.splits * q.npad, u);
}

// Batched max of the block maxima into a scalar slot of each problem.
__global__ void __launch_bounds__(256) k_max_final_b(const BProb *__restrict__ P, BWork w, int64_t out_off)
{
    __shared__ double red[256];
    const BProb &q = P[w.plist[blockIdx.x]];
    const Plan pl = plan_for(q.n);
    const double *blkmax = q.partial + pl.splits * q.npad;
    const int64_t nb = q.npad / 256;
    double v = 0.0;
    for (int64_t e = threadIdx.x; e < nb; e += 256) v = fmax(v, blkmax[e]);
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s2]);
        __syncthreads();
    }
    if (threadIdx.x == 0) q.scal[out_off] = red[0];
}

}  // namespace

size_t zmv_partial_doubles(int64_t n)
{
    Plan p = plan_for(n);
    return (size_t)(p.splits * p.npad + p.npad / 256 + 8);
}

int64_t zmv_b_units(int64_t n)
{
    Plan p = plan_for(n);
    return p.rowblocks * p.splits;
}

// Batched y_slot = Z v_slot (mode 0) or y_slot = b - Z v_slot with its max norm
// into vec[norm_off] (mode 1).  wz: units zmv_b_units(n); wr: units npad/256.
void launch_zmv_b(hipStream_t s, int m, const BProb *P, const BWork &wz, const BWork &wr,
                  int v_slot, int y_slot, int b_slot, int mode, int64_t norm_off)
{
    if (wz.na <= 0) return;
    const dim3 g((unsigned)wz.total);
    switch (m) {
    case 1: hipLaunchKernelGGL(k_zmv_partial_b<1>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    case 2: hipLaunchKernelGGL(k_zmv_partial_b<2>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    case 3: hipLaunchKernelGGL(k_zmv_partial_b<3>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    case 4: hipLaunchKernelGGL(k_zmv_partial_b<4>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    case 8: hipLaunchKernelGGL(k_zmv_partial_b<8>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    default: hipLaunchKernelGGL(k_zmv_partial_b<0>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    }
    hipLaunchKernelGGL(k_zmv_reduce_b, dim3((unsigned)wr.total), dim3(256), 0, s, P, wr, y_slot,
                       b_slot, mode);
    if (mode == 1)
        hipLaunchKernelGGL(k_max_final_b, dim3(wz.na), dim3(256), 0, s, P, wz, norm_off);
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
