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

__global__ void k_scale(const double *x, double a, double *y, int64_t n, int64_t len)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (i < n) ? a * x[i] : 0.0;
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
void launch_scale(hipStream_t s, const double *x, double a, double *y, int64_t n, int64_t len)
{
    hipLaunchKernelGGL(k_scale, dim3(grid_for(len)), dim3(256), 0, s, x, a, y, n, len);
}

size_t blas1_partial_doubles(int kmax) { return (size_t)RG * (size_t)(kmax > 3 ? kmax : 3); }

}  // namespace mag
