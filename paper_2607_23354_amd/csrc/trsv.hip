// trsv.hip -- preconditioner apply z = L^{-T} L^{-1} r of the refinement, and
// the substitution of the FP64 dense factor.
//
// L is the FP32 Cholesky factor (column-major, leading dimension npad, lower
// triangle), r and z are FP64 and all arithmetic is FP64.  The diagonal
// 128 x 128 blocks are applied through their explicit inverses (FP32, from the
// factorisation), so a block step is a small matrix-vector product.  Two
// kernels share the hand-off protocol below:
//   * the band kernel (trsv_body, one workgroup per two blocks) serves the
//     batched solves and, instantiated for the FP64 factor, its 64 x 64 blocks
//     (whose FP64 inverses fit LDS); the figures below are those of the FP32
//     factor at n = 32768;
//   * k_trsv1 (one workgroup per block, composite near step, further down)
//     serves the single FP32 solves: 0.58 ms per direction at n = 32768
//     against the band kernel's 0.97 ms.
//
// Each triangular solve is ONE launch and no host round trips ("sync-free"
// substitution).  For the band kernel:
//   * a workgroup owns a band of two consecutive blocks and takes a ticket
//     from an atomic counter; ticket order is the band order of the
//     substitution, so every block a workgroup waits for belongs to a
//     workgroup that is already running -- forward progress does not depend
//     on how many workgroups fit on the device;
//   * block b streams its off-diagonal tiles in order (forward: L(b, j) from
//     the lower triangle; backward: L^T(b, j) from the upper triangle, where
//     the factorisation keeps the transpose); the tiles of a pair of outside
//     blocks are loaded into registers a whole pair-step ahead of the wait
//     for the solution blocks they multiply, and the band's own right-hand
//     side and inner tile before the first wait, so the HBM stream stays off
//     the dependency chain.  What stays on it, per band (measured at
//     n = 32768 with in-kernel clock stamps, 7.2 us per band): 2.9 us from a
//     band's last store to the next band seeing it, 1.3 us for the four FP64
//     tile products with the received blocks (FP64-FMA bound: 64 Ki products
//     and conversions on one CU), 2.7 us for the two diagonal solves, the
//     inner tile and the LDS reductions;
//   * the solution vector is the flag: before a solve every entry holds an
//     "unset" bit pattern (a signalling NaN no arithmetic produces); a band
//     writes its solution entries with relaxed agent-scope atomic stores, and
//     a waiting band's wave 0 reads the entries it needs with relaxed
//     agent-scope atomic loads until none is unset.  Each entry is written
//     once, so a value that is not the pattern is final: no counter, no
//     release or acquire fence (each fence a wave executes costs microseconds
//     of L2 write-back or invalidation) and no second read of the data;
//   * wave 0 alone polls and copies the received blocks into LDS for the
//     others;
//   * spin-waits are bounded: on exhaustion the kernel sets a status word and
//     finishes, and the host reports an error.
// HBM traffic per apply: the lower triangle read twice (n^2 * 4 bytes).
#include "internal.hpp"

namespace mag {
namespace {

constexpr int kSlot = 64;  // ints between the two tickets (256 bytes)

// counter layout (ints): fwd ticket @0, bwd ticket @kSlot
constexpr int kFwdTicket = 0;
constexpr int kBwdTicket = kSlot;
constexpr int kCounterInts = 2 * kSlot;

// the "unset" entry: a signalling NaN payload (arithmetic yields quiet NaNs)
constexpr uint64_t kUnset = 0x7ff4dead0badf00dull;

__device__ inline uint64_t ld_entry(const double *x, int64_t i)
{
    return __hip_atomic_load(reinterpret_cast<const uint64_t *>(x) + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void st_entry(double *x, int64_t i, double v)
{
    __hip_atomic_store(reinterpret_cast<uint64_t *>(x) + i, __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Wave 0 (lanes 0..63): wait until the BS entries of block j0 (and j1 if two)
// of x are set, and copy them to xs[0] (xs[1]).  Bounded: after spin_limit
// polls the status word is set and whatever was read is used.
template <int BS>
__device__ inline void wait_blocks(const double *x, int64_t j0, int64_t j1, bool two, double (&xs)[2][BS],
                                   int *status, long spin_limit)
{
    static_assert(BS == 64 || BS == 128, "one or two entries per lane and block");
    constexpr bool E2 = BS == 128;
    const int lane = threadIdx.x;
    uint64_t a0, a1 = 0, c0 = 0, c1 = 0;
    long spins = 0;
    for (;;) {
        a0 = ld_entry(x, j0 * BS + lane);
        if (E2) a1 = ld_entry(x, j0 * BS + lane + 64);
        if (two) {
            c0 = ld_entry(x, j1 * BS + lane);
            if (E2) c1 = ld_entry(x, j1 * BS + lane + 64);
        }
        const bool miss = a0 == kUnset || (E2 && a1 == kUnset) || (two && (c0 == kUnset || (E2 && c1 == kUnset)));
        if (__ballot(miss) == 0) break;
        if (++spins > spin_limit) {
            if (lane == 0) status[kStSpinTimeout] = 1;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    xs[0][lane] = __builtin_bit_cast(double, a0);
    if (E2) xs[0][lane + 64] = __builtin_bit_cast(double, a1);
    if (two) {
        xs[1][lane] = __builtin_bit_cast(double, c0);
        if (E2) xs[1][lane + 64] = __builtin_bit_cast(double, c1);
    }
}

// Four consecutive factor entries (one row group of a tile column).
template <typename T>
struct Quad {
    T v[4];
};
__device__ inline void load_quad(const float *p, Quad<float> &q)
{
    const float4 f = *reinterpret_cast<const float4 *>(p);
    q.v[0] = f.x;
    q.v[1] = f.y;
    q.v[2] = f.z;
    q.v[3] = f.w;
}
__device__ inline void load_quad(const double *p, Quad<double> &q)
{
    const double2 a = *reinterpret_cast<const double2 *>(p);
    const double2 b = *reinterpret_cast<const double2 *>(p + 2);
    q.v[0] = a.x;
    q.v[1] = a.y;
    q.v[2] = b.x;
    q.v[3] = b.y;
}

// One triangular solve.  Forward (BWD = false): y = L^{-1} r, block b pulls
// tiles L(b, j), j < b, from the lower triangle.  Backward (BWD = true):
// z = L^{-T} y, block b pulls tiles L^T(b, j), j > b, from the upper
// triangle, where the factorisation stored L^T.  Both read a BS-row band of
// column segments per step, the same HBM access pattern.
//
// A workgroup owns two consecutive blocks (a 2 BS-row band): it streams both
// blocks' tiles against every finished block outside the band, then solves
// the first block, applies the band's inner tile and solves the second, so
// the dependency chain crosses workgroups once per 2 BS rows.
// T, BS: the FP32 factor with 128-blocks, or the FP64 factor with 64-blocks.
template <bool BWD, typename T, int BS>
__device__ __forceinline__ void trsv_body(const T *__restrict__ L, int64_t ld,
                                          const T *__restrict__ dinv,
                                          const double *__restrict__ rhs, double *__restrict__ x,
                                          int *counters, int nblk, int *status, long spin_limit)
{
    constexpr int RG = BS / 4;      // row groups of a tile (4 rows each)
    constexpr int CG = 256 / RG;    // column groups
    constexpr int CPG = BS / CG;    // columns per group
    constexpr int H = 256 / BS;     // parts of a diagonal-block row's product
    constexpr int HC = BS / H;      // columns per part
    static_assert(RG * CG == 256 && CG * CPG == BS && H <= CG, "tile mapping");
    __shared__ T Dl[2][BS * (BS + 1)];  // Dinv of the two blocks, row-major, padded stride
    __shared__ double xs[2][BS];
    __shared__ double part[CG][BS];     // per column group partial sums of a block's rows
    __shared__ int s_band;
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
    // tile products: thread (rg, cg) owns rows 4 rg .. 4 rg + 3 and columns
    // CPG cg .. CPG cg + CPG - 1 of a BS x BS tile (four entries per column)
    const int rg = tid % RG, cg = tid / RG;
    // block solves: thread (h, row) takes part h of row's dot product
    const int row = tid % BS;
    const int h = tid / BS;

    // tile (b, j): element (r, c) at L[(j BS + c) ld + b BS + r] -- forward L(b, j)
    // from the lower triangle, backward L^T(b, j) from the upper triangle
    using Tile = Quad<T>[CPG];
    auto load = [&](int b, int j, Tile &t) {
        const T *p = L + ((int64_t)j * BS + CPG * cg) * ld + (int64_t)b * BS + 4 * rg;
#pragma unroll
        for (int c = 0; c < CPG; ++c) load_quad(p + (int64_t)c * ld, t[c]);
    };
    auto gemv = [&](const Tile &t, const double *xv, double (&acc)[4]) {
#pragma unroll
        for (int c = 0; c < CPG; ++c) {
            const double v = xv[CPG * cg + c];
            acc[0] += (double)t[c].v[0] * v;
            acc[1] += (double)t[c].v[1] * v;
            acc[2] += (double)t[c].v[2] * v;
            acc[3] += (double)t[c].v[3] * v;
        }
    };

    // the right-hand side of both blocks and the band's inner tile (b1, b0) do not
    // depend on other bands: fetch them first, off the dependency chain
    double rhs0 = 0.0, rhs1 = 0.0;
    if (tid < BS) {
        rhs0 = rhs[(int64_t)b0 * BS + tid];
        rhs1 = rhs[(int64_t)b1 * BS + tid];
    }
    Tile ti;
    load(b1, b0, ti);

    // Dinv (column-major in memory) into row-major padded LDS
    for (int q = 0; q < 2; ++q) {
        const T *src = dinv + (int64_t)(q == 0 ? b0 : b1) * BS * BS;
        for (int e = tid; e < BS * BS; e += 256) {
            const int rr = e % BS, cc = e / BS;
            Dl[q][rr * (BS + 1) + cc] = src[e];
        }
    }
    double acc0[4] = {0.0, 0.0, 0.0, 0.0}, acc1[4] = {0.0, 0.0, 0.0, 0.0};
    // blocks outside the band, in the order they finish, two at a time.  A
    // pair's tiles are fetched before its wait, the next pair's right after it.
    const int nsteps = BWD ? (nblk - 2 - 2 * band) : 2 * band;
    Tile ta0, ta1, tb0, tb1;
    auto jof = [&](int st) { return BWD ? (nblk - 1 - st) : st; };
    // steps st and st + 1 (if any): wave 0 waits for both solution blocks (a
    // band writes its two blocks moments apart) and copies them to LDS
    auto consume2 = [&](int st, bool two) {
        if (tid < 64) wait_blocks<BS>(x, jof(st), two ? jof(st + 1) : 0, two, xs, status, spin_limit);
        __syncthreads();
        gemv(ta0, xs[0], acc0);
        gemv(ta1, xs[0], acc1);
        if (two) {
            gemv(tb0, xs[1], acc0);
            gemv(tb1, xs[1], acc1);
        }
        // xs is rewritten by the next step; after the last one, only once the
        // partial sums have passed the next barrier
        if (st + 2 < nsteps) __syncthreads();
    };
    if (nsteps > 0) {
        load(b0, jof(0), ta0);
        load(b1, jof(0), ta1);
    }
    if (nsteps > 1) {
        load(b0, jof(1), tb0);
        load(b1, jof(1), tb1);
    }
    for (int st = 0; st < nsteps; st += 2) {
        const bool two = st + 1 < nsteps;
        consume2(st, two);
        // both tiles of the next pair, a whole step ahead of their wait
        if (st + 2 < nsteps) {
            load(b0, jof(st + 2), ta0);
            load(b1, jof(st + 2), ta1);
        }
        if (st + 3 < nsteps) {
            load(b0, jof(st + 3), tb0);
            load(b1, jof(st + 3), tb1);
        }
    }

    // first block: x_b0 = Dinv_b0 (rhs_b0 - acc0)   (backward: Dinv^T)
#pragma unroll
    for (int i = 0; i < 4; ++i) part[cg][4 * rg + i] = acc0[i];
    __syncthreads();
    if (tid < BS) {
        double sacc = 0.0;
#pragma unroll
        for (int g = 0; g < CG; ++g) sacc += part[g][tid];
        xs[0][tid] = rhs0 - sacc;
    }
    __syncthreads();
    double v = 0.0;
#pragma unroll 16
    for (int c = 0; c < HC; ++c) {
        const int cc = h * HC + c;
        const T d = BWD ? Dl[0][cc * (BS + 1) + row] : Dl[0][row * (BS + 1) + cc];
        v += (double)d * xs[0][cc];
    }
    part[h][row] = v;
    __syncthreads();
    if (tid < BS) {
        double sv = part[0][tid];
#pragma unroll
        for (int g = 1; g < H; ++g) sv += part[g][tid];
        xs[1][tid] = sv;
    }
    __syncthreads();
    // wave 0 writes the band's solution entries (each write releases that entry)
    if (tid < 64) {
#pragma unroll
        for (int e = 0; e < BS / 64; ++e) st_entry(x, (int64_t)b0 * BS + tid + 64 * e, xs[1][tid + 64 * e]);
    }
    // second block: acc1 += L(b1, b0) x_b0, then x_b1 = Dinv_b1 (rhs_b1 - acc1)
    gemv(ti, xs[1], acc1);
#pragma unroll
    for (int i = 0; i < 4; ++i) part[cg][4 * rg + i] = acc1[i];
    __syncthreads();
    if (tid < BS) {
        double sacc = 0.0;
#pragma unroll
        for (int g = 0; g < CG; ++g) sacc += part[g][tid];
        xs[0][tid] = rhs1 - sacc;
    }
    __syncthreads();
    v = 0.0;
#pragma unroll 16
    for (int c = 0; c < HC; ++c) {
        const int cc = h * HC + c;
        const T d = BWD ? Dl[1][cc * (BS + 1) + row] : Dl[1][row * (BS + 1) + cc];
        v += (double)d * xs[0][cc];
    }
    part[h][row] = v;
    __syncthreads();
    if (tid < 64) {
#pragma unroll
        for (int e = 0; e < BS / 64; ++e) {
            const int rr = tid + 64 * e;
            double sv = part[0][rr];
#pragma unroll
            for (int g = 1; g < H; ++g) sv += part[g][rr];
            st_entry(x, (int64_t)b1 * BS + rr, sv);
        }
    }
}

template <bool BWD, typename T, int BS>
__global__ void __launch_bounds__(256)
k_trsv(const T *__restrict__ L, int64_t ld, const T *__restrict__ dinv,
       const double *__restrict__ rhs, double *__restrict__ x, int *counters, int nblk,
       int *status, long spin_limit)
{
    trsv_body<BWD, T, BS>(L, ld, dinv, rhs, x, counters, nblk, status, spin_limit);
}

// One triangular solve of the FP32 factor with one 128-row block per
// workgroup and a composite near step.  With the solve's block b, its
// predecessor n (b - 1 forward, b + 1 backward) and the blocks before that
// ("far", streamed two at a time as in trsv_body):
//   x_b = y - Q_b x_n,   y = D_b (rhs_b - sum_far T(b, j) x_j),   Q_b = D_b T(b, n),
// with D_b the block's inverse (transposed backward) and T the streamed tile
// (forward L(b, j) from the lower triangle, backward L^T(b, j) from the upper
// one).  Q_b (k_near_q) and D_b stay resident from the workgroup's start, y is
// formed once the far blocks are in, so after its predecessor's block arrives
// a workgroup applies one resident tile and one reduction: the dependency
// chain costs one hand-off and one 128 x 128 product per block.
template <bool BWD>
__device__ __forceinline__ void trsv1_body(const float *__restrict__ L, int64_t ld, const float *__restrict__ dinv,
                                           const float *__restrict__ Qb, const double *__restrict__ rhs,
                                           double *__restrict__ x, int *counters, int nblk, int *status,
                                           long spin_limit)
{
    constexpr int BS = 128;
    __shared__ float Dl[BS * (BS + 1)];  // D_b, row-major, padded stride
    __shared__ double xs[2][BS];
    __shared__ double part[8][BS];
    __shared__ int s_blk;
    const int tid = threadIdx.x;
    if (tid == 0) {
        const int ticket = atomicAdd(&counters[BWD ? kBwdTicket : kFwdTicket], 1);
        s_blk = BWD ? nblk - 1 - ticket : ticket;
    }
    __syncthreads();
    const int b = s_blk;
    const int rg = tid & 31, cg = tid >> 5;     // tile products: rows 4 rg .., columns 16 cg ..
    const int row = tid & (BS - 1), h = tid >> 7;  // block product: half h of row's sum
    using Tile = Quad<float>[16];
    auto load = [&](const float *base, int64_t ldb, Tile &t) {
        const float *p = base + (int64_t)(16 * cg) * ldb + 4 * rg;
#pragma unroll
        for (int c = 0; c < 16; ++c) load_quad(p + (int64_t)c * ldb, t[c]);
    };
    auto tile = [&](int j) { return L + (int64_t)j * BS * ld + (int64_t)b * BS; };
    auto gemv = [&](const Tile &t, const double *xv, double (&acc)[4]) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const double v = xv[16 * cg + c];
            acc[0] += (double)t[c].v[0] * v;
            acc[1] += (double)t[c].v[1] * v;
            acc[2] += (double)t[c].v[2] * v;
            acc[3] += (double)t[c].v[3] * v;
        }
    };
    auto jof = [&](int st) { return BWD ? (nblk - 1 - st) : st; };
    const int nsteps = BWD ? (nblk - 1 - b) : b;  // blocks solved before this one
    const bool has_near = nsteps >= 1;
    const int nfar = has_near ? nsteps - 1 : 0;

    // resident from the start: the right-hand side, D_b and the near tile Q_b
    double r0 = 0.0;
    if (tid < BS) r0 = rhs[(int64_t)b * BS + tid];
    Tile tq;
    if (has_near) load(Qb + (int64_t)b * BS * BS, BS, tq);
    {
        const float *src = dinv + (int64_t)b * BS * BS;
        for (int e = tid; e < BS * BS; e += 256) {
            const int rr = e & (BS - 1), cc = e >> 7;
            Dl[rr * (BS + 1) + cc] = src[e];
        }
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    Tile ta, tb;
    if (nfar > 0) load(tile(jof(0)), ld, ta);
    if (nfar > 1) load(tile(jof(1)), ld, tb);
    for (int st = 0; st < nfar; st += 2) {
        const bool two = st + 1 < nfar;
        if (tid < 64) wait_blocks<BS>(x, jof(st), two ? jof(st + 1) : 0, two, xs, status, spin_limit);
        __syncthreads();
        gemv(ta, xs[0], acc);
        if (two) gemv(tb, xs[1], acc);
        __syncthreads();  // xs is rewritten by the next wait (or the block product below)
        if (st + 2 < nfar) load(tile(jof(st + 2)), ld, ta);
        if (st + 3 < nfar) load(tile(jof(st + 3)), ld, tb);
    }
    // y = D_b (rhs_b - acc)
#pragma unroll
    for (int i = 0; i < 4; ++i) part[cg][4 * rg + i] = acc[i];
    __syncthreads();
    if (tid < BS) {
        double sacc = 0.0;
#pragma unroll
        for (int g = 0; g < 8; ++g) sacc += part[g][tid];
        xs[0][tid] = r0 - sacc;
    }
    __syncthreads();
    double v = 0.0;
#pragma unroll 16
    for (int c = 0; c < 64; ++c) {
        const int cc = h * 64 + c;
        const float d = BWD ? Dl[cc * (BS + 1) + row] : Dl[row * (BS + 1) + cc];
        v += (double)d * xs[0][cc];
    }
    part[h][row] = v;
    __syncthreads();
    double y = 0.0;
    if (tid < BS) y = part[0][tid] + part[1][tid];
    if (!has_near) {
        if (tid < BS) st_entry(x, (int64_t)b * BS + tid, y);
        return;
    }
    // the predecessor's block: x_b = y - Q_b x_n
    __syncthreads();  // part is rewritten below
    if (tid < 64) wait_blocks<BS>(x, jof(nsteps - 1), 0, false, xs, status, spin_limit);
    __syncthreads();
    double aq[4] = {0.0, 0.0, 0.0, 0.0};
    gemv(tq, xs[0], aq);
#pragma unroll
    for (int i = 0; i < 4; ++i) part[cg][4 * rg + i] = aq[i];
    __syncthreads();
    if (tid < BS) {
        double sq = 0.0;
#pragma unroll
        for (int g = 0; g < 8; ++g) sq += part[g][tid];
        st_entry(x, (int64_t)b * BS + tid, y - sq);
    }
}

template <bool BWD>
__global__ void __launch_bounds__(256)
k_trsv1(const float *__restrict__ L, int64_t ld, const float *__restrict__ dinv, const float *__restrict__ Qb,
        const double *__restrict__ rhs, double *__restrict__ x, int *counters, int nblk, int *status,
        long spin_limit)
{
    trsv1_body<BWD>(L, ld, dinv, Qb, rhs, x, counters, nblk, status, spin_limit);
}

// The near tiles of k_trsv1 for every 128-block of the FP32 factor, both
// directions: workgroup (b, d) forms Q = D_b T(b, n) (forward: D_b L(b, b - 1);
// backward: D_b^T L^T(b, b + 1)) with FP64 accumulation of the FP32 entries,
// stored in FP32, column-major, at Q + (d nblk + b) 128^2.  The first block in
// solve order has none.
__global__ void __launch_bounds__(256)
k_near_q(const float *__restrict__ A, int64_t npad, const float *__restrict__ dinv, float *__restrict__ Q, int nblk)
{
    constexpr int B = 128;
    __shared__ float Xs[B * B];  // X(i, k) at Xs[k B + i]
    __shared__ float Ys[B * B];  // Y(k, j) at Ys[k B + j]
    const int b = blockIdx.x, d = blockIdx.y;
    const bool bwd = d == 1;
    if (bwd ? (b >= nblk - 1) : (b == 0)) return;  // uniform per workgroup
    const int jn = bwd ? b + 1 : b - 1;
    const int tid = threadIdx.x;
    const int ti = tid & 15, tj = tid >> 4;  // output rows 8 ti .., columns 8 tj ..
    const float *D = dinv + (int64_t)b * B * B;  // column-major inverse
    for (int e = tid; e < B * B; e += 256) {
        const int i = e & (B - 1), k = e >> 7;
        Xs[k * B + i] = bwd ? D[i * B + k] : D[k * B + i];
        // tile T(b, jn): element (r, c) at A[(jn B + c) npad + b B + r], as Y(k = r, j = c)
        Ys[i * B + k] = A[((int64_t)jn * B + k) * npad + (int64_t)b * B + i];
    }
    __syncthreads();
    double acc[8][8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[a][c] = 0.0;
    for (int k = 0; k < B; ++k) {
        const float4 xa = *reinterpret_cast<const float4 *>(&Xs[k * B + 8 * ti]);
        const float4 xb = *reinterpret_cast<const float4 *>(&Xs[k * B + 8 * ti + 4]);
        const float4 ya = *reinterpret_cast<const float4 *>(&Ys[k * B + 8 * tj]);
        const float4 yb = *reinterpret_cast<const float4 *>(&Ys[k * B + 8 * tj + 4]);
        const double xv[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
        const double yv[8] = {ya.x, ya.y, ya.z, ya.w, yb.x, yb.y, yb.z, yb.w};
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[a][c] = fma(xv[a], yv[c], acc[a][c]);
    }
    float *dst = Q + ((int64_t)d * nblk + b) * B * B;
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int a = 0; a < 8; ++a) dst[(8 * tj + c) * B + 8 * ti + a] = (float)acc[a][c];
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
    trsv_body<BWD, float, 128>(q.A, q.npad, q.dinv, q.vec + (int64_t)rhs_slot * q.npad,
                               q.vec + (int64_t)x_slot * q.npad, q.ints + 64, (int)(q.npad / 128), q.ints,
                               kSpinLimitDefault);
}

// Tickets to zero and the vector in `slot` unset, one workgroup per problem
// (tickets: only when `tickets`).
__global__ void k_unset_b(const BProb *__restrict__ P, BWork w, int slot, int tickets)
{
    const BProb &q = P[w.plist[blockIdx.x]];
    if (!q.active) return;
    if (tickets)
        for (int e = threadIdx.x; e < kCounterInts; e += blockDim.x) q.ints[64 + e] = 0;
    uint64_t *a = reinterpret_cast<uint64_t *>(q.vec + (int64_t)slot * q.npad);
    for (int64_t e = threadIdx.x; e < q.npad; e += blockDim.x) a[e] = kUnset;
}

// Every entry of a (n entries) unset.
__global__ void k_unset(double *__restrict__ a, int64_t n)
{
    uint64_t *u = reinterpret_cast<uint64_t *>(a);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        u[e] = kUnset;
}

}  // namespace

size_t prec_counter_ints() { return kCounterInts; }

int64_t prec_b_units(int64_t npad) { return npad / 256; }

// x_slot = (L L^T)^{-1} rhs_slot for every problem of the work list (units = npad/128 each)
void launch_prec_apply_b(hipStream_t s, const BProb *P, const BWork &w, int rhs_slot, int tmp_slot,
                         int x_slot)
{
    if (w.na <= 0) return;
    hipLaunchKernelGGL(k_unset_b, dim3(w.na), dim3(256), 0, s, P, w, tmp_slot, 1);
    hipLaunchKernelGGL(k_trsv_b<false>, dim3((unsigned)w.total), dim3(256), 0, s, P, w, rhs_slot, tmp_slot);
    hipLaunchKernelGGL(k_unset_b, dim3(w.na), dim3(256), 0, s, P, w, x_slot, 0);
    hipLaunchKernelGGL(k_trsv_b<true>, dim3((unsigned)w.total), dim3(256), 0, s, P, w, tmp_slot, x_slot);
}

template <typename T, int BS>
void prec_apply(hipStream_t s, const T *L, int64_t npad, const T *dinv, const double *r, double *y_tmp, double *z,
                int *counters, int *status, long spin_limit)
{
    const int nblk = (int)(npad / BS);  // even: npad is a multiple of 256
    const unsigned gu = (unsigned)std::min<int64_t>((npad + 255) / 256, 1024);
    launch_fill_ints(s, counters, kCounterInts, 0);
    hipLaunchKernelGGL(k_unset, dim3(gu), dim3(256), 0, s, y_tmp, npad);
    hipLaunchKernelGGL((k_trsv<false, T, BS>), dim3(nblk / 2), dim3(256), 0, s, L, npad, dinv, r, y_tmp, counters,
                       nblk, status, spin_limit);
    // z may be the caller's r: unset it only once the forward solve has read r
    hipLaunchKernelGGL(k_unset, dim3(gu), dim3(256), 0, s, z, npad);
    hipLaunchKernelGGL((k_trsv<true, T, BS>), dim3(nblk / 2), dim3(256), 0, s, L, npad, dinv, y_tmp, z, counters,
                       nblk, status, spin_limit);
}

void launch_prec_apply(hipStream_t s, const float *L, int64_t npad, const float *dinv,
                       const double *r, double *y_tmp, double *z, int *counters, int *status, const float *Q,
                       long spin_limit)
{
    const int nblk = (int)(npad / 128);
    const float *Qb = Q + (int64_t)nblk * 128 * 128;  // the backward direction's tiles
    const unsigned gu = (unsigned)std::min<int64_t>((npad + 255) / 256, 1024);
    launch_fill_ints(s, counters, kCounterInts, 0);
    hipLaunchKernelGGL(k_unset, dim3(gu), dim3(256), 0, s, y_tmp, npad);
    hipLaunchKernelGGL(k_trsv1<false>, dim3(nblk), dim3(256), 0, s, L, npad, dinv, Q, r, y_tmp, counters, nblk,
                       status, spin_limit);
    // z may be the caller's r: unset it only once the forward solve has read r
    hipLaunchKernelGGL(k_unset, dim3(gu), dim3(256), 0, s, z, npad);
    hipLaunchKernelGGL(k_trsv1<true>, dim3(nblk), dim3(256), 0, s, L, npad, dinv, Qb, y_tmp, z, counters, nblk,
                       status, spin_limit);
}

size_t near_q_floats(int64_t npad) { return (size_t)npad * 256; }

void launch_near_q(hipStream_t s, const float *A, int64_t npad, const float *dinv, float *Q)
{
    const int nblk = (int)(npad / 128);
    if (nblk < 2) return;
    hipLaunchKernelGGL(k_near_q, dim3((unsigned)nblk, 2), dim3(256), 0, s, A, npad, dinv, Q, nblk);
}

void launch_chol64_solve(hipStream_t s, const double *L, int64_t npad, const double *dinv, const double *r,
                         double *y_tmp, double *z, int *counters, int *status,
                        long spin_limit)
{
    prec_apply<double, 64>(s, L, npad, dinv, r, y_tmp, z, counters, status, spin_limit);
}

}  // namespace mag
