// trsv.hip -- preconditioner apply z = L^{-T} L^{-1} r of the refinement.
//
// L is the FP32 Cholesky factor (column-major, leading dimension npad, lower
// triangle), r and z are FP64 and all arithmetic is FP64.  The diagonal
// 128 x 128 blocks are applied through their explicit inverses (FP32, from the
// factorisation), so a block step is a small matrix-vector product.
//
// Each triangular solve is ONE launch with one workgroup per 128-row block
// and no host round trips ("sync-free" substitution):
//   * a workgroup takes a ticket from an atomic counter; ticket order is the
//     block order of the substitution, so every block a workgroup waits for
//     belongs to a workgroup that is already running -- forward progress
//     does not depend on how many workgroups fit on the device;
//   * block b streams its off-diagonal tiles L(b, j), j < b, as soon as the
//     corresponding solution blocks are published; a single "ready" counter
//     (blocks [0, ready) are final) replaces per-block flags, since block b
//     can only finish after block b-1 has;
//   * publication is a release store of the counter after an agent-scope
//     fence; consumers read it with acquire loads, which also invalidate
//     stale lines of other XCDs' L2.
// Spin-waits are bounded: on exhaustion the kernel sets a status word and
// finishes, and the host reports an error.
// The HBM traffic per apply is the lower triangle read twice (n^2 * 4 bytes).
#include "internal.hpp"

namespace mag {
namespace {

constexpr int BS = 128;
constexpr long kSpinLimit = 1L << 25;

enum { kFwdTicket = 0, kFwdReady = 1, kBwdTicket = 2, kBwdReady = 3, kCounters = 4 };

__device__ inline int wait_ready(int *ready, int need, int *status)
{
    int v;
    long spins = 0;
    while ((v = __hip_atomic_load(ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) < need) {
        if (++spins > kSpinLimit) {
            status[kStSpinTimeout] = 1;
            return 1 << 30;  // give up: treat everything as ready
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return v;
}

__global__ void __launch_bounds__(256)
k_trsv_fwd(const float *__restrict__ L, int64_t ld, const float *__restrict__ dinv,
           const double *__restrict__ r, double *__restrict__ y, int *counters, int nblk,
           int *status)
{
    __shared__ double ys[BS];
    __shared__ double part[2][BS];
    __shared__ int s_b, s_ready;
    const int tid = threadIdx.x;
    if (tid == 0) s_b = atomicAdd(&counters[kFwdTicket], 1);
    __syncthreads();
    const int b = s_b;
    const int row = tid & (BS - 1);
    const int h = tid >> 7;
    double acc = 0.0;
    int known = 0;
    for (int j = 0; j < b; ++j) {
        if (j >= known) {
            if (tid == 0) s_ready = wait_ready(&counters[kFwdReady], j + 1, status);
            __syncthreads();
            known = s_ready;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (tid < BS) ys[tid] = y[(int64_t)j * BS + tid];
        __syncthreads();
        const float *Lt = L + ((int64_t)j * BS + h * 64) * ld + (int64_t)b * BS + row;
#pragma unroll 16
        for (int c = 0; c < 64; ++c) acc += (double)Lt[(int64_t)c * ld] * ys[h * 64 + c];
        __syncthreads();
    }
    part[h][row] = acc;
    __syncthreads();
    if (tid < BS) ys[tid] = r[(int64_t)b * BS + tid] - (part[0][tid] + part[1][tid]);
    __syncthreads();
    // y_b = Dinv_b * rhs
    const float *D = dinv + (int64_t)b * BS * BS;
    double v = 0.0;
#pragma unroll 16
    for (int c = 0; c < 64; ++c) v += (double)D[(h * 64 + c) * BS + row] * ys[h * 64 + c];
    part[h][row] = v;
    __syncthreads();
    if (tid < BS) y[(int64_t)b * BS + tid] = part[0][tid] + part[1][tid];
    __threadfence();
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&counters[kFwdReady], b + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Reduce a per-lane value over the 64 lanes of a wave.
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(256)
k_trsv_bwd(const float *__restrict__ L, int64_t ld, const float *__restrict__ dinv,
           const double *__restrict__ y, double *__restrict__ z, int *counters, int nblk,
           int *status)
{
    __shared__ double zs[BS];
    __shared__ double part[BS];
    __shared__ int s_b, s_ready;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (tid == 0) s_b = nblk - 1 - atomicAdd(&counters[kBwdTicket], 1);
    __syncthreads();
    const int b = s_b;
    // wave w owns columns 32w .. 32w+31 of the block column b; lane covers rows lane, lane+64
    double acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = 0.0;
    int known = 0;  // blocks nblk-known .. nblk-1 are final
    for (int j = nblk - 1; j > b; --j) {
        const int need = nblk - j;
        if (need > known) {
            if (tid == 0) s_ready = wait_ready(&counters[kBwdReady], need, status);
            __syncthreads();
            known = s_ready;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (tid < BS) zs[tid] = z[(int64_t)j * BS + tid];
        __syncthreads();
        const double z0 = zs[lane], z1 = zs[lane + 64];
        const float *Lt = L + ((int64_t)b * BS + 32 * wave) * ld + (int64_t)j * BS + lane;
#pragma unroll
        for (int c = 0; c < 32; ++c)
            acc[c] += (double)Lt[(int64_t)c * ld] * z0 + (double)Lt[(int64_t)c * ld + 64] * z1;
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        const double s = wave_sum(acc[c]);
        if (lane == 0) part[32 * wave + c] = s;
    }
    __syncthreads();
    if (tid < BS) zs[tid] = y[(int64_t)b * BS + tid] - part[tid];
    __syncthreads();
    // z_b = Dinv_b^T * rhs : z_b[c] = sum_rr Dinv(rr, c) rhs[rr]
    const float *D = dinv + (int64_t)b * BS * BS;
    const double r0 = zs[lane], r1 = zs[lane + 64];
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        const int col = 32 * wave + c;
        double v = (double)D[col * BS + lane] * r0 + (double)D[col * BS + lane + 64] * r1;
        v = wave_sum(v);
        if (lane == 0) part[col] = v;
    }
    __syncthreads();
    if (tid < BS) z[(int64_t)b * BS + tid] = part[tid];
    __threadfence();
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&counters[kBwdReady], nblk - b, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

size_t prec_counter_ints() { return kCounters; }

void launch_prec_apply(hipStream_t s, const float *L, int64_t npad, const float *dinv,
                       const double *r, double *y_tmp, double *z, int *counters, int *status)
{
    const int nblk = (int)(npad / BS);
    launch_fill_ints(s, counters, kCounters, 0);
    hipLaunchKernelGGL(k_trsv_fwd, dim3(nblk), dim3(256), 0, s, L, npad, dinv, r, y_tmp, counters,
                       nblk, status);
    hipLaunchKernelGGL(k_trsv_bwd, dim3(nblk), dim3(256), 0, s, L, npad, dinv, y_tmp, z, counters,
                       nblk, status);
}

}  // namespace mag
