// trsv.hip -- preconditioner apply z = L^{-T} L^{-1} r of the refinement.
//
// L is the FP32 Cholesky factor (column-major, leading dimension npad, lower
// triangle), r and z are FP64 and all arithmetic is FP64.  The diagonal
// 128 x 128 blocks are applied through their explicit inverses (FP32, from the
// factorisation), so a block step is a small matrix-vector product.
//
// Each triangular solve is ONE launch with one workgroup per 128-row block
// and no host round trips ("sync-free" substitution):
//   * a workgroup owns a band of two consecutive blocks and takes a ticket
//     from an atomic counter; ticket order is the band order of the
//     substitution, so every block a workgroup waits for belongs to a
//     workgroup that is already running -- forward progress does not depend
//     on how many workgroups fit on the device;
//   * block b streams its off-diagonal tiles in order (forward: L(b, j) from
//     the lower triangle; backward: L^T(b, j) from the upper triangle, where
//     the factorisation keeps the transpose); the tile is
//     loaded into registers before waiting for the solution block it
//     multiplies, so the HBM stream overlaps the dependency chain;
//   * a "ready" count (blocks [0, ready) are final) replaces per-block flags,
//     since block b can only finish after block b-1 has; a band publishes
//     both of its blocks at once.  It is published in
//     8 mirrored slots 256 bytes apart (each workgroup polls one), with a
//     release after an agent-scope fence of the solution writes; pollers use
//     relaxed loads and take one acquire fence per observed advance (an
//     acquire per poll would invalidate the L2 on every spin);
//   * spin-waits are bounded: on exhaustion the kernel sets a status word and
//     finishes, and the host reports an error.
// HBM traffic per apply: the lower triangle read twice (n^2 * 4 bytes).
#include "internal.hpp"

namespace mag {
namespace {

constexpr int BS = 128;
constexpr long kSpinLimit = 1L << 26;
constexpr int kMirrors = 8;
constexpr int kSlot = 64;  // ints between mirrored slots (256 bytes)

// counter layout (ints): fwd ticket @0, bwd ticket @kSlot,
// fwd ready mirrors @(2+q)*kSlot, bwd ready mirrors @(2+kMirrors+q)*kSlot
constexpr int kFwdTicket = 0;
constexpr int kBwdTicket = kSlot;
constexpr int kFwdReady = 2 * kSlot;
constexpr int kBwdReady = (2 + kMirrors) * kSlot;
constexpr int kCounterInts = (2 + 2 * kMirrors) * kSlot;

__device__ inline int wait_ready(int *ready, int need, int *status)
{
    int v;
    long spins = 0;
    while ((v = __hip_atomic_load(ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < need) {
        if (++spins > kSpinLimit) {
            status[kStSpinTimeout] = 1;
            return 1 << 30;  // give up: treat everything as ready
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return v;
}

__device__ inline void publish(int *base, int value)
{
    // every thread fenced its own solution writes before the barrier
    if (threadIdx.x < kMirrors)
        __hip_atomic_store(base + threadIdx.x * kSlot, value, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// One triangular solve.  Forward (BWD = false): y = L^{-1} r, block b pulls
// tiles L(b, j), j < b, from the lower triangle.  Backward (BWD = true):
// z = L^{-T} y, block b pulls tiles L^T(b, j), j > b, from the upper
// triangle, where the factorisation stored L^T.  Both read a 128-row band of
// 512-byte column segments per step, the same HBM access pattern.
//
// A workgroup owns two consecutive blocks (a 256-row band): it streams both
// blocks' tiles against every finished block outside the band, then solves
// the first block, applies the band's inner tile and solves the second, so
// the dependency chain crosses workgroups once per 256 rows.
template <bool BWD>
__device__ __forceinline__ void trsv_body(const float *__restrict__ L, int64_t ld,
                                          const float *__restrict__ dinv,
                                          const double *__restrict__ rhs, double *__restrict__ x,
                                          int *counters, int nblk, int *status)
{
    __shared__ float Dl[2][BS * (BS + 1)];  // Dinv of the two blocks, row-major, padded stride
    __shared__ double xs[2][BS];
    __shared__ double part[2][2][BS];
    __shared__ int s_band, s_ready;
    const int tid = threadIdx.x;
    const int nband = nblk / 2;
    if (tid == 0) {
        const int ticket = atomicAdd(&counters[BWD ? kBwdTicket : kFwdTicket], 1);
        s_band = BWD ? nband - 1 - ticket : ticket;
    }
    __syncthreads();
    const int band = s_band;
    // blocks in solve order: forward (2 band, 2 band + 1), backward (2 band + 1, 2 band)
    const int b0 = BWD ? 2 * band + 1 : 2 * band;
    const int b1 = BWD ? 2 * band : 2 * band + 1;
    const int row = tid & (BS - 1);
    const int h = tid >> 7;
    int *ready = counters + (BWD ? kBwdReady : kFwdReady) + (band % kMirrors) * kSlot;

    // Dinv (column-major in memory) into row-major padded LDS
    for (int q = 0; q < 2; ++q) {
        const float *src = dinv + (int64_t)(q == 0 ? b0 : b1) * BS * BS;
        for (int e = tid; e < BS * BS; e += 256) {
            const int rr = e & (BS - 1), cc = e >> 7;
            Dl[q][rr * (BS + 1) + cc] = src[e];
        }
    }
    double acc0 = 0.0, acc1 = 0.0;
    int known = 0;
    // blocks outside the band, in the order they finish; ready counts finished blocks
    const int nsteps = BWD ? (nblk - 2 - 2 * band) : 2 * band;
    for (int s = 0; s < nsteps; ++s) {
        const int j = BWD ? (nblk - 1 - s) : s;
        float lt0[64], lt1[64];
        const float *L0 = L + ((int64_t)j * BS + h * 64) * ld + (int64_t)b0 * BS + row;
        const float *L1 = L + ((int64_t)j * BS + h * 64) * ld + (int64_t)b1 * BS + row;
#pragma unroll
        for (int c = 0; c < 64; ++c) {
            lt0[c] = L0[(int64_t)c * ld];
            lt1[c] = L1[(int64_t)c * ld];
        }
        if (s >= known) {
            if (tid == 0) s_ready = wait_ready(ready, s + 1, status);
            __syncthreads();
            known = s_ready;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        double *xb = xs[s & 1];
        if (tid < BS) xb[tid] = x[(int64_t)j * BS + tid];
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 64; ++c) {
            const double xv = xb[h * 64 + c];
            acc0 += (double)lt0[c] * xv;
            acc1 += (double)lt1[c] * xv;
        }
    }
    // the band's inner tile (b1, b0), loaded while the first block is solved
    float lti[64];
    {
        const float *Li = L + ((int64_t)b0 * BS + h * 64) * ld + (int64_t)b1 * BS + row;
#pragma unroll
        for (int c = 0; c < 64; ++c) lti[c] = Li[(int64_t)c * ld];
    }
    part[0][h][row] = acc0;
    part[1][h][row] = acc1;
    __syncthreads();
    // first block: x_b0 = Dinv_b0 (rhs_b0 - acc0)   (backward: Dinv^T)
    if (tid < BS) xs[0][tid] = rhs[(int64_t)b0 * BS + tid] - (part[0][0][tid] + part[0][1][tid]);
    __syncthreads();
    double v = 0.0;
#pragma unroll 16
    for (int c = 0; c < 64; ++c) {
        const int cc = h * 64 + c;
        const float d = BWD ? Dl[0][cc * (BS + 1) + row] : Dl[0][row * (BS + 1) + cc];
        v += (double)d * xs[0][cc];
    }
    part[0][h][row] = v;
    __syncthreads();
    if (tid < BS) {
        const double xv = part[0][0][tid] + part[0][1][tid];
        xs[1][tid] = xv;
        x[(int64_t)b0 * BS + tid] = xv;
    }
    __syncthreads();
    // second block: acc1 += L(b1, b0) x_b0, then x_b1 = Dinv_b1 (rhs_b1 - acc1)
#pragma unroll
    for (int c = 0; c < 64; ++c) acc1 += (double)lti[c] * xs[1][h * 64 + c];
    part[1][h][row] = acc1;
    __syncthreads();
    if (tid < BS) xs[0][tid] = rhs[(int64_t)b1 * BS + tid] - (part[1][0][tid] + part[1][1][tid]);
    __syncthreads();
    v = 0.0;
#pragma unroll 16
    for (int c = 0; c < 64; ++c) {
        const int cc = h * 64 + c;
        const float d = BWD ? Dl[1][cc * (BS + 1) + row] : Dl[1][row * (BS + 1) + cc];
        v += (double)d * xs[0][cc];
    }
    part[1][h][row] = v;
    __syncthreads();
    if (tid < BS) x[(int64_t)b1 * BS + tid] = part[1][0][tid] + part[1][1][tid];
    __threadfence();
    __syncthreads();
    publish(counters + (BWD ? kBwdReady : kFwdReady), nsteps + 2);
}

template <bool BWD>
__global__ void __launch_bounds__(256)
k_trsv(const float *__restrict__ L, int64_t ld, const float *__restrict__ dinv,
       const double *__restrict__ rhs, double *__restrict__ x, int *counters, int nblk,
       int *status)
{
    trsv_body<BWD>(L, ld, dinv, rhs, x, counters, nblk, status);
}

// Batched: workgroups of problem p take tickets from p's own counters, so the
// forward-progress argument holds per problem; problems never wait on each other.
template <bool BWD>
__global__ void __launch_bounds__(256)
k_trsv_b(const BProb *__restrict__ P, BWork w, int rhs_slot, int x_slot)
{
    const int i = bfind(w.pref, w.na, blockIdx.x);
    const BProb &q = P[w.plist[i]];
    if (!q.active) return;
    trsv_body<BWD>(q.A, q.npad, q.dinv, q.vec + (int64_t)rhs_slot * q.npad,
                   q.vec + (int64_t)x_slot * q.npad, q.ints + 64, (int)(q.npad / BS), q.ints);
}

__global__ void k_zero_counters_b(const BProb *__restrict__ P, BWork w)
{
    const BProb &q = P[w.plist[blockIdx.x]];
    for (int e = threadIdx.x; e < kCounterInts; e += blockDim.x) q.ints[64 + e] = 0;
}

}  // namespace

size_t prec_counter_ints() { return kCounterInts; }

int64_t prec_b_units(int64_t npad) { return npad / (2 * BS); }

// x_slot = (L L^T)^{-1} rhs_slot for every problem of the work list (units = npad/128 each)
void launch_prec_apply_b(hipStream_t s, const BProb *P, const BWork &w, int rhs_slot, int tmp_slot,
                         int x_slot)
{
    if (w.na <= 0) return;
    hipLaunchKernelGGL(k_zero_counters_b, dim3(w.na), dim3(256), 0, s, P, w);
    hipLaunchKernelGGL(k_trsv_b<false>, dim3((unsigned)w.total), dim3(256), 0, s, P, w, rhs_slot, tmp_slot);
    hipLaunchKernelGGL(k_trsv_b<true>, dim3((unsigned)w.total), dim3(256), 0, s, P, w, tmp_slot, x_slot);
}

void launch_prec_apply(hipStream_t s, const float *L, int64_t npad, const float *dinv,
                       const double *r, double *y_tmp, double *z, int *counters, int *status)
{
    const int nblk = (int)(npad / BS);  // even: npad is a multiple of 256
    launch_fill_ints(s, counters, kCounterInts, 0);
    hipLaunchKernelGGL(k_trsv<false>, dim3(nblk / 2), dim3(256), 0, s, L, npad, dinv, r, y_tmp, counters,
                       nblk, status);
    hipLaunchKernelGGL(k_trsv<true>, dim3(nblk / 2), dim3(256), 0, s, L, npad, dinv, y_tmp, z, counters,
                       nblk, status);
}

}  // namespace mag
