// pairwise.hip -- matrix-free FP64 passes over all pairs (j, k) for the
// derivatives of the weighting.  Differentiating Z(t, X) w = 1 (Section 2,
// eq. weighting) with Z_jk = exp(-t d_jk):
//   dZ_jk/dt     = -d_jk Z_jk                        -> (D o Z) v  (kDZ)
//   dZ_jk/dx_j   = -t Z_jk (x_j - x_k) / d_jk        -> gradient   (kGradX)
// so, with lambda = Z^{-1}(gM 1 + gw):
//   dL/dt   = lambda^T (D o Z) w
//   dL/dx_j = t sum_{k != j} (lambda_j w_k + lambda_k w_j) Z_jk (x_j - x_k) / d_jk.
// Entries are formed exactly as the tile generator forms Z (exact
// differences, uncontracted squared sum, sqrt, exp(-(t d))).  Same grid as
// the Z v product: row blocks x column splits, split partials reduced in a
// fixed order.
#include "internal.hpp"

#include <cmath>

namespace mag {
namespace {

constexpr int RT = 256;
constexpr int CH = 256;
constexpr int MMAX = 16;  // largest dimension of the register-held forms

__device__ inline double sq_acc(double s, double e)
{
#pragma clang fp contract(off)
    double p = e * e;
    return s + p;
}

enum { kDZ = 0, kGradX = 1 };

// M > 0: compile-time dimension; M == 0: runtime m <= MMAX.
template <int MODE, int M>
__device__ __forceinline__ void pair_partial_body(const double *__restrict__ X, int64_t n, int m_rt,
                                                  double t, const double *__restrict__ v,
                                                  const double *__restrict__ lam,
                                                  double *__restrict__ partial, int64_t cps,
                                                  int64_t npad, int64_t bx, int64_t by)
{
    constexpr int MM = (M > 0) ? M : MMAX;
    __shared__ double Xc[MM * CH];
    __shared__ double vc[CH];
    __shared__ double lc[CH];
    const int m = (M > 0) ? M : m_rt;
    const int64_t j = bx * RT + threadIdx.x;
    const int64_t c_lo = by * cps;
    const int64_t c_hi = min(n, c_lo + cps);
    const bool live = j < n;
    double xr[MM];
    double acc[MODE == kGradX ? MM : 1];
#pragma unroll
    for (int l = 0; l < MM; ++l) xr[l] = (live && l < m) ? X[j * m + l] : 0.0;
#pragma unroll
    for (int l = 0; l < (MODE == kGradX ? MM : 1); ++l) acc[l] = 0.0;
    const double vj = live ? v[j] : 0.0;
    const double lj = (MODE == kGradX && live) ? lam[j] : 0.0;

    for (int64_t k0 = c_lo; k0 < c_hi; k0 += CH) {
        const int cnt = (int)min((int64_t)CH, c_hi - k0);
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * m; e += RT) {
            const int p = e / m, l = e % m;
            Xc[l * CH + p] = X[(k0 + p) * m + l];
        }
        if (threadIdx.x < cnt) {
            vc[threadIdx.x] = v[k0 + threadIdx.x];
            if (MODE == kGradX) lc[threadIdx.x] = lam[k0 + threadIdx.x];
        }
        __syncthreads();
        if (!live) continue;
        for (int c = 0; c < cnt; ++c) {
            if (k0 + c == j) continue;
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < MM; ++l)
                if (l < m) s = sq_acc(s, xr[l] - Xc[l * CH + c]);
            const double d = sqrt(s);
            const double z = exp_nonpos(-(t * d));
            if (MODE == kDZ) {
                acc[0] = fma(d * z, vc[c], acc[0]);
            } else {
                const double coef = t * (lj * vc[c] + lc[c] * vj) * z / d;
#pragma unroll
                for (int l = 0; l < MM; ++l)
                    if (l < m) acc[l] = fma(coef, xr[l] - Xc[l * CH + c], acc[l]);
            }
        }
    }
    if (j < npad) {
        if (MODE == kDZ) {
            partial[by * npad + j] = live ? acc[0] : 0.0;
        } else {
#pragma unroll
            for (int l = 0; l < MM; ++l)
                if (l < m) partial[(by * npad + j) * m + l] = live ? acc[l] : 0.0;
        }
    }
}

// Any m (used above MMAX): each thread reads its own row and the column points
// from global memory (L1/L2 cached); the gradient's m outputs are formed in
// passes of GCH dimensions, each pass recomputing the entries over all m.
constexpr int GCH = 16;

template <int MODE>
__device__ __forceinline__ void pair_partial_generic(const double *__restrict__ X, int64_t n, int m, double t,
                                                     const double *__restrict__ v,
                                                     const double *__restrict__ lam,
                                                     double *__restrict__ partial, int64_t cps, int64_t npad,
                                                     int64_t bx, int64_t by)
{
    __shared__ double vc[CH];
    __shared__ double lc[CH];
    const int64_t j = bx * RT + threadIdx.x;
    const int64_t c_lo = by * cps;
    const int64_t c_hi = min(n, c_lo + cps);
    const bool live = j < n;
    const double vj = live ? v[j] : 0.0;
    const double lj = (MODE == kGradX && live) ? lam[j] : 0.0;
    const double *xj = X + (live ? j : 0) * m;
    const int passes = (MODE == kGradX) ? (m + GCH - 1) / GCH : 1;
    for (int pass = 0; pass < passes; ++pass) {
        const int l0 = pass * GCH;
        double acc[GCH];
#pragma unroll
        for (int q = 0; q < GCH; ++q) acc[q] = 0.0;
        for (int64_t k0 = c_lo; k0 < c_hi; k0 += CH) {
            const int cnt = (int)min((int64_t)CH, c_hi - k0);
            __syncthreads();
            if (threadIdx.x < cnt) {
                vc[threadIdx.x] = v[k0 + threadIdx.x];
                if (MODE == kGradX) lc[threadIdx.x] = lam[k0 + threadIdx.x];
            }
            __syncthreads();
            if (!live) continue;
            for (int c = 0; c < cnt; ++c) {
                if (k0 + c == j) continue;
                const double *xk = X + (k0 + c) * m;
                double s = 0.0;
                for (int l = 0; l < m; ++l) s = sq_acc(s, xj[l] - xk[l]);
                const double d = sqrt(s);
                const double z = exp_nonpos(-(t * d));
                if (MODE == kDZ) {
                    acc[0] = fma(d * z, vc[c], acc[0]);
                } else {
                    const double coef = t * (lj * vc[c] + lc[c] * vj) * z / d;
#pragma unroll
                    for (int q = 0; q < GCH; ++q)
                        if (l0 + q < m) acc[q] = fma(coef, xj[l0 + q] - xk[l0 + q], acc[q]);
                }
            }
        }
        if (j < npad) {
            if (MODE == kDZ) {
                partial[by * npad + j] = live ? acc[0] : 0.0;
            } else {
#pragma unroll
                for (int q = 0; q < GCH; ++q)
                    if (l0 + q < m) partial[(by * npad + j) * m + l0 + q] = live ? acc[q] : 0.0;
            }
        }
    }
}

template <int MODE>
__global__ void __launch_bounds__(RT)
k_pair_partial_generic(const double *__restrict__ X, int64_t n, int m, double t, const double *__restrict__ v,
                       const double *__restrict__ lam, double *__restrict__ partial, int64_t cps, int64_t npad)
{
    pair_partial_generic<MODE>(X, n, m, t, v, lam, partial, cps, npad, blockIdx.x, blockIdx.y);
}

template <int MODE, int M>
__global__ void __launch_bounds__(RT)
k_pair_partial(const double *__restrict__ X, int64_t n, int m_rt, double t,
               const double *__restrict__ v, const double *__restrict__ lam,
               double *__restrict__ partial, int64_t cps, int64_t npad)
{
    pair_partial_body<MODE, M>(X, n, m_rt, t, v, lam, partial, cps, npad, blockIdx.x, blockIdx.y);
}

// out[e] = sum_s partial[s * stride + e] for e < count (fixed order)
__global__ void k_split_reduce(const double *__restrict__ partial, int64_t stride, int splits,
                               int64_t count, double *__restrict__ out)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < splits; ++q) s += partial[(int64_t)q * stride + e];
        out[e] = s;
    }
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

// Batched (D o Z) v: units rowblocks * splits per problem, then a reduce over
// the splits (units npad/256 per problem).
template <int M>
__global__ void __launch_bounds__(RT) k_dz_partial_b(const BProb *__restrict__ P, BWork w, int v_slot)
{
    const int i = bfind(w.pref, w.na, blockIdx.x);
    const BProb &q = P[w.plist[i]];
    if (!q.active) return;
    const Plan pl = plan_for(q.n);
    const int64_t u = blockIdx.x - w.pref[i];
    pair_partial_body<kDZ, M>(q.X, q.n, q.m, q.t, q.vec + (int64_t)v_slot * q.npad, nullptr,
                              q.partial, pl.cps, q.npad, u / pl.splits, u % pl.splits);
}

__global__ void __launch_bounds__(RT) k_dz_partial_generic_b(const BProb *__restrict__ P, BWork w, int v_slot)
{
    const int i = bfind(w.pref, w.na, blockIdx.x);
    const BProb &q = P[w.plist[i]];
    if (!q.active) return;
    const Plan pl = plan_for(q.n);
    const int64_t u = blockIdx.x - w.pref[i];
    pair_partial_generic<kDZ>(q.X, q.n, q.m, q.t, q.vec + (int64_t)v_slot * q.npad, nullptr, q.partial, pl.cps,
                              q.npad, u / pl.splits, u % pl.splits);
}

__global__ void __launch_bounds__(256) k_dz_reduce_b(const BProb *__restrict__ P, BWork w, int y_slot)
{
    const int i = bfind(w.pref, w.na, blockIdx.x);
    const BProb &q = P[w.plist[i]];
    if (!q.active) return;
    const Plan pl = plan_for(q.n);
    const int64_t j = (blockIdx.x - w.pref[i]) * 256 + threadIdx.x;
    if (j >= q.npad) return;
    double s = 0.0;
    for (int k = 0; k < pl.splits; ++k) s += q.partial[k * q.npad + j];
    q.vec[(int64_t)y_slot * q.npad + j] = s;
}

template <int MODE>
void launch_mode(hipStream_t s, const Plan &p, dim3 grid, const double *X, int64_t n, int m,
                 double t, const double *v, const double *lam, double *partial)
{
#define MAG_PAIR_CASE(MV)                                                                        \
    hipLaunchKernelGGL((k_pair_partial<MODE, MV>), grid, dim3(RT), 0, s, X, n, m, t, v, lam,     \
                       partial, p.cps, p.npad)
    switch (m) {
    case 1: MAG_PAIR_CASE(1); break;
    case 2: MAG_PAIR_CASE(2); break;
    case 3: MAG_PAIR_CASE(3); break;
    case 4: MAG_PAIR_CASE(4); break;
    case 8: MAG_PAIR_CASE(8); break;
    default:
        if (m <= MMAX) MAG_PAIR_CASE(0);
        else hipLaunchKernelGGL(k_pair_partial_generic<MODE>, grid, dim3(RT), 0, s, X, n, m, t, v, lam, partial,
                                p.cps, p.npad);
        break;
    }
#undef MAG_PAIR_CASE
}

}  // namespace

// Every pass accepts any dimension (compile-time forms up to MMAX, the generic
// form above); the bound only guards the int arithmetic of the layouts.
int pair_max_dim() { return 1 << 16; }

int64_t dz_b_units(int64_t n)
{
    Plan p = plan_for(n);
    return p.rowblocks * p.splits;
}

void launch_dzmv_b(hipStream_t s, int m, const BProb *P, const BWork &wz, const BWork &wr,
                   int v_slot, int y_slot)
{
    if (wz.na <= 0) return;
    const dim3 g((unsigned)wz.total);
    switch (m) {
    case 1: hipLaunchKernelGGL(k_dz_partial_b<1>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    case 2: hipLaunchKernelGGL(k_dz_partial_b<2>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    case 3: hipLaunchKernelGGL(k_dz_partial_b<3>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    case 4: hipLaunchKernelGGL(k_dz_partial_b<4>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    case 8: hipLaunchKernelGGL(k_dz_partial_b<8>, g, dim3(RT), 0, s, P, wz, v_slot); break;
    default:
        if (m <= MMAX) hipLaunchKernelGGL(k_dz_partial_b<0>, g, dim3(RT), 0, s, P, wz, v_slot);
        else hipLaunchKernelGGL(k_dz_partial_generic_b, g, dim3(RT), 0, s, P, wz, v_slot);
        break;
    }
    hipLaunchKernelGGL(k_dz_reduce_b, dim3((unsigned)wr.total), dim3(256), 0, s, P, wr, y_slot);
}

size_t pair_partial_doubles(int64_t n, int m)
{
    Plan p = plan_for(n);
    return (size_t)(p.splits * p.npad * (m > 1 ? m : 1));
}

// y (npad) = (D o Z) v
void launch_dzmv(hipStream_t s, const double *X, int64_t n, int m, double t, const double *v,
                 double *y, double *partial)
{
    Plan p = plan_for(n);
    dim3 grid((unsigned)p.rowblocks, (unsigned)p.splits);
    launch_mode<kDZ>(s, p, grid, X, n, m, t, v, nullptr, partial);
    hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((p.npad + 255) / 256)), dim3(256), 0, s,
                       partial, p.npad, (int)p.splits, p.npad, y);
}

// dX (n x m, row-major) = t sum_{k != j} (lam_j w_k + lam_k w_j) Z_jk (x_j - x_k) / d_jk
void launch_gradx(hipStream_t s, const double *X, int64_t n, int m, double t, const double *w,
                  const double *lam, double *dX, double *partial)
{
    Plan p = plan_for(n);
    dim3 grid((unsigned)p.rowblocks, (unsigned)p.splits);
    launch_mode<kGradX>(s, p, grid, X, n, m, t, w, lam, partial);
    const int64_t cnt = n * (int64_t)m;
    int64_t blocks = (cnt + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)blocks), dim3(256), 0, s, partial,
                       p.npad * m, (int)p.splits, cnt, dX);
}

}  // namespace mag
