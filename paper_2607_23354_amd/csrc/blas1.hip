// blas1.hip -- FP64 vector kernels of the refinement loop (GMRES Arnoldi
// steps, norms, the magnitude sum and the minimum weight).  Every reduction
// is two-pass with a fixed order, so results are bitwise reproducible.
#include "internal.hpp"

#include <cmath>

namespace mag {
namespace {

constexpr int RB = 256;     // threads per reduction block
constexpr int RG = 128;     // reduction blocks (first pass)

__device__ inline double block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

__global__ void k_fill(double *x, int64_t len, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_fill_ints(int *x, int64_t len, int v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_copy(const double *x, double *y, int64_t len)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i];
}

__global__ void k_axpy1(const double *x, double *y, int64_t len)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] += x[i];
}

__global__ void k_scale_inv(const double *x, double *y, int64_t len, const double *alpha)
{
    const double a = 1.0 / alpha[0];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i] * a;
}

// partial[i * RG + g] = sum over chunk g of V_i . u
__global__ void __launch_bounds__(RB)
k_multidot_partial(const double *V, int64_t ld, const double *u, int64_t len, double *partial)
{
    __shared__ double red[RB];
    const int i = blockIdx.y;
    const int g = blockIdx.x;
    const double *vi = V + (int64_t)i * ld;
    const int64_t chunk = (len + RG - 1) / RG;
    const int64_t lo = g * chunk, hi = min(len, lo + chunk);
    double s = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += RB) s = fma(vi[e], u[e], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[(int64_t)i * RG + g] = s;
}

__global__ void __launch_bounds__(RB) k_rows_sum(const double *partial, int k, double *out)
{
    __shared__ double red[RB];
    for (int i = 0; i < k; ++i) {
        double s = (threadIdx.x < RG) ? partial[(int64_t)i * RG + threadIdx.x] : 0.0;
        s = block_sum(s, red);
        if (threadIdx.x == 0) out[i] = s;
    }
}

__global__ void k_multi_axpy(const double *V, int64_t ld, int k, const double *h, double *u,
                             int64_t len, double sign)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s = fma(h[i], V[(int64_t)i * ld + e], s);
        u[e] = fma(sign, s, u[e]);
    }
}

__global__ void __launch_bounds__(RB) k_sumsq_partial(const double *x, int64_t len, double *partial)
{
    __shared__ double red[RB];
    const int64_t chunk = (len + RG - 1) / RG;
    const int64_t lo = blockIdx.x * chunk, hi = min(len, lo + chunk);
    double s = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += RB) s = fma(x[e], x[e], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(RB) k_sqrt_sum(const double *partial, double *out)
{
    __shared__ double red[RB];
    double s = (threadIdx.x < RG) ? partial[threadIdx.x] : 0.0;
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[0] = sqrt(s);
}

// partial[3g] = sum, [3g+1] = min, [3g+2] = argmin (as double) over chunk g
__global__ void __launch_bounds__(RB) k_summin_partial(const double *x, int64_t n, double *partial)
{
    __shared__ double red[RB];
    __shared__ double rmin[RB];
    __shared__ int64_t rarg[RB];
    const int64_t chunk = (n + RG - 1) / RG;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double s = 0.0, mn = INFINITY;
    int64_t am = -1;
    for (int64_t e = lo + threadIdx.x; e < hi; e += RB) {
        const double v = x[e];
        s += v;
        if (v < mn) { mn = v; am = e; }
    }
    rmin[threadIdx.x] = mn;
    rarg[threadIdx.x] = am;
    s = block_sum(s, red);  // contains barriers
    for (int w = RB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double a = rmin[threadIdx.x], b = rmin[threadIdx.x + w];
            const int64_t ia = rarg[threadIdx.x], ib = rarg[threadIdx.x + w];
            if (b < a || (b == a && ib >= 0 && (ia < 0 || ib < ia))) {
                rmin[threadIdx.x] = b;
                rarg[threadIdx.x] = ib;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x] = s;
        partial[3 * blockIdx.x + 1] = rmin[0];
        partial[3 * blockIdx.x + 2] = (double)rarg[0];
    }
}

__global__ void k_summin_final(const double *partial, double *out)
{
    if (threadIdx.x != 0) return;
    double s = 0.0, c = 0.0, mn = INFINITY, am = -1.0;
    for (int g = 0; g < RG; ++g) {
        // Neumaier-compensated accumulation of the block sums
        const double x = partial[3 * g];
        const double u = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - u) + x) : ((x - u) + s);
        s = u;
        const double v = partial[3 * g + 1];
        const double a = partial[3 * g + 2];
        if (v < mn || (v == mn && a >= 0 && (am < 0 || a < am))) { mn = v; am = a; }
    }
    out[0] = s + c;
    out[1] = mn;
    out[2] = am;
}

__global__ void __launch_bounds__(RB) k_amax_partial(const double *x, int64_t len, double *partial)
{
    __shared__ double red[RB];
    const int64_t chunk = (len + RG - 1) / RG;
    const int64_t lo = blockIdx.x * chunk, hi = min(len, lo + chunk);
    double s = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += RB) s = fmax(s, fabs(x[e]));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(RB) k_amax_final(const double *partial, double *out)
{
    __shared__ double red[RB];
    red[threadIdx.x] = (threadIdx.x < RG) ? partial[threadIdx.x] : 0.0;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// y[j] = a + (x ? x[j] : 0) for j < n, 0 for n <= j < len
__global__ void k_affine_ones(const double *x, double a, double *y, int64_t n, int64_t len)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (i < n) ? a + (x ? x[i] : 0.0) : 0.0;
}

// Deterministic start vector with no special structure: the Weyl sequence of
// the golden ratio, shifted to (1/2, 3/2).
__global__ void k_golden(double *y, int64_t n, int64_t len)
{
    const double g = 0.6180339887498949;  // (sqrt 5 - 1) / 2
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (i < n) {
            const double p = (double)(i + 1) * g;
            v = 0.5 + (p - floor(p));
        }
        y[i] = v;
    }
}

__global__ void k_scale(const double *x, double a, double *y, int64_t n, int64_t len)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (i < n) ? a * x[i] : 0.0;
}

// ---- batched forms: blockIdx.y = work item, problem plist[blockIdx.y] --------
// Vectors are slots of length npad in each problem's q.vec; scalars live in
// q.scal.

__global__ void k_fill_b(const BProb *__restrict__ P, const int *plist, int slot, double v, int upto_n)
{
    const BProb &q = P[plist[blockIdx.y]];
    if (!q.active) return;
    double *x = q.vec + (int64_t)slot * q.npad;
    const int64_t len = upto_n ? q.n : q.npad;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q.npad;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = (i < len) ? v : 0.0;
}

__global__ void k_copy_b(const BProb *__restrict__ P, const int *plist, int src, int dst)
{
    const BProb &q = P[plist[blockIdx.y]];
    if (!q.active) return;
    const double *x = q.vec + (int64_t)src * q.npad;
    double *y = q.vec + (int64_t)dst * q.npad;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q.npad;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i];
}

// y = x / vec[scal_off]
__global__ void k_scale_inv_b(const BProb *__restrict__ P, const int *plist, int src, int dst,
                              int64_t scal_off)
{
    const BProb &q = P[plist[blockIdx.y]];
    if (!q.active) return;
    const double a = 1.0 / q.scal[scal_off];
    const double *x = q.vec + (int64_t)src * q.npad;
    double *y = q.vec + (int64_t)dst * q.npad;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q.npad;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i] * a;
}

// partial (per problem, q.partial) [j * RG + g] = chunk g of V_j . u, V_j = slot v0 + j
__global__ void __launch_bounds__(RB)
k_multidot_partial_b(const BProb *__restrict__ P, const int *plist, int v0, int k, int u_slot)
{
    __shared__ double red[RB];
    const BProb &q = P[plist[blockIdx.y]];
    if (!q.active) return;
    const int g = blockIdx.x;
    const int64_t len = q.npad;
    const double *u = q.vec + (int64_t)u_slot * len;
    const int64_t chunk = (len + RG - 1) / RG;
    const int64_t lo = g * chunk, hi = min(len, lo + chunk);
    for (int j = 0; j < k; ++j) {
        const double *vj = q.vec + (int64_t)(v0 + j) * len;
        double s = 0.0;
        for (int64_t e = lo + threadIdx.x; e < hi; e += RB) s = fma(vj[e], u[e], s);
        s = block_sum(s, red);
        if (threadIdx.x == 0) q.partial[(int64_t)j * RG + g] = s;
    }
}

// vec[out_off + j] = sum_g partial[j * RG + g], j < k
__global__ void __launch_bounds__(RB) k_rows_sum_b(const BProb *__restrict__ P, const int *plist, int k,
                                                    int64_t out_off)
{
    __shared__ double red[RB];
    const BProb &q = P[plist[blockIdx.x]];
    if (!q.active) return;
    for (int j = 0; j < k; ++j) {
        double s = (threadIdx.x < RG) ? q.partial[(int64_t)j * RG + threadIdx.x] : 0.0;
        s = block_sum(s, red);
        if (threadIdx.x == 0) q.scal[out_off + j] = s;
    }
}

// u += sign * sum_j vec[h_off + j] * V_j
__global__ void k_multi_axpy_b(const BProb *__restrict__ P, const int *plist, int v0, int k,
                               int64_t h_off, int u_slot, double sign)
{
    const BProb &q = P[plist[blockIdx.y]];
    if (!q.active) return;
    const double *h = q.scal + h_off;
    double *u = q.vec + (int64_t)u_slot * q.npad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < q.npad;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s = fma(h[j], q.vec[(int64_t)(v0 + j) * q.npad + e], s);
        u[e] = fma(sign, s, u[e]);
    }
}

// u += sign * sum_j hb[i * k + j] * V_j for work item i (coefficients in one array)
__global__ void k_multi_axpy_hb(const BProb *__restrict__ P, const int *plist, int v0, int k,
                                const double *hb, int u_slot, double sign)
{
    const BProb &q = P[plist[blockIdx.y]];
    if (!q.active) return;
    const double *h = hb + (int64_t)blockIdx.y * k;
    double *u = q.vec + (int64_t)u_slot * q.npad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < q.npad;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s = fma(h[j], q.vec[(int64_t)(v0 + j) * q.npad + e], s);
        u[e] = fma(sign, s, u[e]);
    }
}

__global__ void __launch_bounds__(RB) k_nrm2_b(const BProb *__restrict__ P, const int *plist, int slot,
                                                int64_t out_off)
{
    // one block per problem (vectors are short in batched use)
    __shared__ double red[RB];
    const BProb &q = P[plist[blockIdx.x]];
    if (!q.active) return;
    const double *x = q.vec + (int64_t)slot * q.npad;
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < q.npad; e += RB) s = fma(x[e], x[e], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) q.scal[out_off] = sqrt(s);
}

// vec[out_off] = sum, [+1] = min, [+2] = argmin of slot[0, n)
__global__ void __launch_bounds__(RB) k_summin_b(const BProb *__restrict__ P, const int *plist, int slot,
                                                  int64_t out_off)
{
    __shared__ double red[RB];
    __shared__ double rmin[RB];
    __shared__ int64_t rarg[RB];
    const BProb &q = P[plist[blockIdx.x]];
    if (!q.active) return;
    const double *x = q.vec + (int64_t)slot * q.npad;
    double s = 0.0, c = 0.0, mn = INFINITY;
    int64_t am = -1;
    for (int64_t e = threadIdx.x; e < q.n; e += RB) {
        const double v = x[e];
        const double u = s + v;  // Neumaier-compensated per-thread sum
        c += (fabs(s) >= fabs(v)) ? ((s - u) + v) : ((v - u) + s);
        s = u;
        if (v < mn) { mn = v; am = e; }
    }
    rmin[threadIdx.x] = mn;
    rarg[threadIdx.x] = am;
    s = block_sum(s + c, red);
    for (int w = RB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double a = rmin[threadIdx.x], b = rmin[threadIdx.x + w];
            const int64_t ia = rarg[threadIdx.x], ib = rarg[threadIdx.x + w];
            if (b < a || (b == a && ib >= 0 && (ia < 0 || ib < ia))) {
                rmin[threadIdx.x] = b;
                rarg[threadIdx.x] = ib;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        q.scal[out_off] = s;
        q.scal[out_off + 1] = rmin[0];
        q.scal[out_off + 2] = (double)rarg[0];
    }
}

__global__ void __launch_bounds__(RB) k_amax_b(const BProb *__restrict__ P, const int *plist, int slot,
                                                int64_t out_off)
{
    __shared__ double red[RB];
    const BProb &q = P[plist[blockIdx.x]];
    if (!q.active) return;
    const double *x = q.vec + (int64_t)slot * q.npad;
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < q.npad; e += RB) s = fmax(s, fabs(x[e]));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) q.scal[out_off] = red[0];
}

__global__ void k_gather_scal_b(const BProb *__restrict__ P, const int *plist, int na, int64_t off,
                                int cnt, double *out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= na * cnt) return;
    const int i = e / cnt, c = e % cnt;
    out[e] = P[plist[i]].scal[off + c];
}

// scal[dst] = vec[slot][(int64_t)scal[idx_off]] (an element picked by a device index)
__global__ void k_pick_b(const BProb *__restrict__ P, const int *plist, int na, int slot, int64_t idx_off,
                         int64_t dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= na) return;
    const BProb &q = P[plist[i]];
    if (!q.active) return;
    const int64_t j = (int64_t)q.scal[idx_off];
    q.scal[dst] = (j >= 0 && j < q.n) ? q.vec[(int64_t)slot * q.npad + j] : 0.0;
}

// zero the status words of each listed problem (graph-safe: a kernel, not a memset)
__global__ void k_zero_status_b(const BProb *__restrict__ P, const int *plist, int na)
{
    const int i = blockIdx.x;
    if (i >= na) return;
    if (threadIdx.x < 64) P[plist[i]].ints[threadIdx.x] = 0;
}

// copy vec slot [0, n) of each listed problem into a packed output at out + offs[i]
__global__ void k_unpack_b(const BProb *__restrict__ P, const int *plist, const int64_t *offs, int slot,
                           double *out)
{
    const BProb &q = P[plist[blockIdx.y]];
    const double *x = q.vec + (int64_t)slot * q.npad;
    double *y = out + offs[blockIdx.y];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < q.n;
         e += (int64_t)gridDim.x * blockDim.x)
        y[e] = x[e];
}

inline unsigned grid_for(int64_t len)
{
    int64_t b = (len + 255) / 256;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

void launch_fill(hipStream_t s, double *x, int64_t len, double v)
{
    hipLaunchKernelGGL(k_fill, dim3(grid_for(len)), dim3(256), 0, s, x, len, v);
}
void launch_fill_ints(hipStream_t s, int *x, int64_t len, int v)
{
    hipLaunchKernelGGL(k_fill_ints, dim3(grid_for(len)), dim3(256), 0, s, x, len, v);
}
void launch_copy(hipStream_t s, const double *x, double *y, int64_t len)
{
    hipLaunchKernelGGL(k_copy, dim3(grid_for(len)), dim3(256), 0, s, x, y, len);
}
void launch_axpy1(hipStream_t s, const double *x, double *y, int64_t len)
{
    hipLaunchKernelGGL(k_axpy1, dim3(grid_for(len)), dim3(256), 0, s, x, y, len);
}
void launch_scale_inv(hipStream_t s, const double *x, double *y, int64_t len, const double *alpha)
{
    hipLaunchKernelGGL(k_scale_inv, dim3(grid_for(len)), dim3(256), 0, s, x, y, len, alpha);
}
void launch_multidot(hipStream_t s, const double *V, int64_t ld, int k, const double *u,
                     int64_t len, double *partial, double *h)
{
    hipLaunchKernelGGL(k_multidot_partial, dim3(RG, k), dim3(RB), 0, s, V, ld, u, len, partial);
    hipLaunchKernelGGL(k_rows_sum, dim3(1), dim3(RB), 0, s, partial, k, h);
}
void launch_multi_axpy(hipStream_t s, const double *V, int64_t ld, int k, const double *h,
                       double *u, int64_t len, double sign)
{
    hipLaunchKernelGGL(k_multi_axpy, dim3(grid_for(len)), dim3(256), 0, s, V, ld, k, h, u, len, sign);
}
void launch_nrm2(hipStream_t s, const double *x, int64_t len, double *partial, double *out)
{
    hipLaunchKernelGGL(k_sumsq_partial, dim3(RG), dim3(RB), 0, s, x, len, partial);
    hipLaunchKernelGGL(k_sqrt_sum, dim3(1), dim3(RB), 0, s, partial, out);
}
void launch_sum_min(hipStream_t s, const double *x, int64_t n, double *partial, double *out)
{
    hipLaunchKernelGGL(k_summin_partial, dim3(RG), dim3(RB), 0, s, x, n, partial);
    hipLaunchKernelGGL(k_summin_final, dim3(1), dim3(64), 0, s, partial, out);
}

void launch_amax(hipStream_t s, const double *x, int64_t len, double *partial, double *out)
{
    hipLaunchKernelGGL(k_amax_partial, dim3(RG), dim3(RB), 0, s, x, len, partial);
    hipLaunchKernelGGL(k_amax_final, dim3(1), dim3(RB), 0, s, partial, out);
}
void launch_affine_ones(hipStream_t s, const double *x, double a, double *y, int64_t n, int64_t len)
{
    hipLaunchKernelGGL(k_affine_ones, dim3(grid_for(len)), dim3(256), 0, s, x, a, y, n, len);
}
void launch_golden(hipStream_t s, double *y, int64_t n, int64_t len)
{
    hipLaunchKernelGGL(k_golden, dim3(grid_for(len)), dim3(256), 0, s, y, n, len);
}
void launch_scale(hipStream_t s, const double *x, double a, double *y, int64_t n, int64_t len)
{
    hipLaunchKernelGGL(k_scale, dim3(grid_for(len)), dim3(256), 0, s, x, a, y, n, len);
}

// ---- batched launchers (na = number of work items, plist on the device) ------
void launch_fill_b(hipStream_t s, const BProb *P, const int *plist, int na, int64_t maxpad, int slot,
                   double v, bool upto_n)
{
    if (na > 0) hipLaunchKernelGGL(k_fill_b, dim3(grid_for(maxpad) > 64 ? 64 : grid_for(maxpad), na),
                                   dim3(256), 0, s, P, plist, slot, v, upto_n ? 1 : 0);
}
void launch_copy_b(hipStream_t s, const BProb *P, const int *plist, int na, int64_t maxpad, int src, int dst)
{
    if (na > 0) hipLaunchKernelGGL(k_copy_b, dim3(grid_for(maxpad) > 64 ? 64 : grid_for(maxpad), na),
                                   dim3(256), 0, s, P, plist, src, dst);
}
void launch_scale_inv_b(hipStream_t s, const BProb *P, const int *plist, int na, int64_t maxpad, int src,
                        int dst, int64_t scal_off)
{
    if (na > 0) hipLaunchKernelGGL(k_scale_inv_b, dim3(grid_for(maxpad) > 64 ? 64 : grid_for(maxpad), na),
                                   dim3(256), 0, s, P, plist, src, dst, scal_off);
}
void launch_multidot_b(hipStream_t s, const BProb *P, const int *plist, int na, int v0, int k, int u_slot,
                       int64_t out_off)
{
    if (na <= 0) return;
    hipLaunchKernelGGL(k_multidot_partial_b, dim3(RG, na), dim3(RB), 0, s, P, plist, v0, k, u_slot);
    hipLaunchKernelGGL(k_rows_sum_b, dim3(na), dim3(RB), 0, s, P, plist, k, out_off);
}
void launch_multi_axpy_b(hipStream_t s, const BProb *P, const int *plist, int na, int64_t maxpad, int v0,
                         int k, int64_t h_off, int u_slot, double sign)
{
    if (na > 0) hipLaunchKernelGGL(k_multi_axpy_b, dim3(grid_for(maxpad) > 64 ? 64 : grid_for(maxpad), na),
                                   dim3(256), 0, s, P, plist, v0, k, h_off, u_slot, sign);
}
void launch_multi_axpy_hb(hipStream_t s, const BProb *P, const int *plist, int na, int64_t maxpad, int v0,
                          int k, const double *hb, int u_slot, double sign)
{
    if (na > 0 && k > 0)
        hipLaunchKernelGGL(k_multi_axpy_hb, dim3(grid_for(maxpad) > 64 ? 64 : grid_for(maxpad), na), dim3(256),
                           0, s, P, plist, v0, k, hb, u_slot, sign);
}
void launch_nrm2_b(hipStream_t s, const BProb *P, const int *plist, int na, int slot, int64_t out_off)
{
    if (na > 0) hipLaunchKernelGGL(k_nrm2_b, dim3(na), dim3(RB), 0, s, P, plist, slot, out_off);
}
void launch_summin_b(hipStream_t s, const BProb *P, const int *plist, int na, int slot, int64_t out_off)
{
    if (na > 0) hipLaunchKernelGGL(k_summin_b, dim3(na), dim3(RB), 0, s, P, plist, slot, out_off);
}
void launch_amax_b(hipStream_t s, const BProb *P, const int *plist, int na, int slot, int64_t out_off)
{
    if (na > 0) hipLaunchKernelGGL(k_amax_b, dim3(na), dim3(RB), 0, s, P, plist, slot, out_off);
}

void launch_gather_scal_b(hipStream_t s, const BProb *P, const int *plist, int na, int64_t off, int cnt,
                          double *out)
{
    const int tot = na * cnt;
    if (tot > 0) hipLaunchKernelGGL(k_gather_scal_b, dim3((tot + 255) / 256), dim3(256), 0, s, P, plist, na, off, cnt, out);
}
void launch_pick_b(hipStream_t s, const BProb *P, const int *plist, int na, int slot, int64_t idx_off,
                   int64_t dst)
{
    if (na > 0) hipLaunchKernelGGL(k_pick_b, dim3((na + 255) / 256), dim3(256), 0, s, P, plist, na, slot, idx_off, dst);
}
void launch_zero_status_b(hipStream_t s, const BProb *P, const int *plist, int na)
{
    if (na > 0) hipLaunchKernelGGL(k_zero_status_b, dim3(na), dim3(64), 0, s, P, plist, na);
}
void launch_unpack_b(hipStream_t s, const BProb *P, const int *plist, int na, const int64_t *offs, int slot,
                     double *out, int64_t maxn)
{
    if (na > 0) hipLaunchKernelGGL(k_unpack_b, dim3(grid_for(maxn) > 64 ? 64 : grid_for(maxn), na), dim3(256), 0,
                                   s, P, plist, offs, slot, out);
}

size_t blas1_partial_doubles(int kmax) { return (size_t)RG * (size_t)(kmax > 3 ? kmax : 3); }

}  // namespace mag
