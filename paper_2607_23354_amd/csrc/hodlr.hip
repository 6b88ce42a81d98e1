// hodlr.hip -- hierarchical off-diagonal low-rank (HODLR) preconditioner for
// Z w = 1 at sizes where a dense factor is not the best tool.
//
// Section 3.2 of the paper solves the weighting system with a hierarchical
// (rank-structured) factorization whose compression step evaluates kernel
// entries and whose factorization step dominates the time.  This file builds
// a HODLR approximation H of Z and its inverse in product form; GMRES with the
// exact FP64 matrix-free Z v (gemv64.hip) then solves Z w = 1 to full
// accuracy, so H only has to be a good preconditioner.
//
// Cluster tree.  Points are ordered by recursive coordinate bisection: each
// node is split at the median of its widest coordinate (ties by index).  The
// tree is perfect with L levels (2^l nodes at level l, leaves at level L,
// every leaf holding at most 256 points); node (l, i) covers the permuted
// index range [bnd_l[i], bnd_l[i+1]).
//
// Off-diagonal blocks.  For node N = (l, i) with children I (left) and J
// (right), Z(I, J) ~ U_I V_J^T with U_I an orthonormal basis of the sample
// Z(I, J) Omega (Omega Gaussian with k_l columns) and V_J = Z(J, I) U_I.  Z
// entries are regenerated in FP64 from the coordinates (exact differences).
// The basis width k_l is a multiple of 64 that shrinks towards the leaves:
// across a cut, the points within the kernel's reach of the other side
// grow with the node, and so does the rank a given accuracy needs.  P_l
// (n x k_l, row-major) holds U_I on the rows of every left child and V_J on
// the rows of every right child.
//
// Inverse in product form.  With D_N = diag(H_I, H_J),
//   H_N = D_N (I + Ut_N Vt_N^T),   Ut_N = diag(H_I^{-1} U_I, H_J^{-1} V_J),
//   Vt_N^T x = [V_J^T x_J ; U_I^T x_I],
//   H_N^{-1} = (I - Ut_N K_N^{-1} Vt_N^T) D_N^{-1},
//   K_N = I + Vt_N^T Ut_N = [[I, B], [C, I]],  B = V_J^T H_J^{-1} V_J,  C = U_I^T H_I^{-1} U_I,
// and K_N^{-1} [s1; s2] = [x1; s2 - C x1] with x1 = (I - B C)^{-1} (s1 - B s2),
// so only the k x k Schur complement S = I - B C is inverted.  Then
// H^{-1} = W_0 W_1 ... W_{L-1} D_L^{-1}, W_l the block-diagonal corrections
// of level l and D_L the exact leaf blocks.  Ph_l holds H_child^{-1} P_l: it
// starts as D_L^{-1} P_l and receives the corrections of every deeper level,
// bottom-up.
//
// Sampling, Gram and row products, leaf inverses of up to 128 points (whole in
// LDS) and the apply are kernels of this file; the per-node k x k algebra
// (Cholesky and triangular inverse of the Gram matrices, the Schur complements
// and their LU inverses, products of k x k blocks) and the batched Cholesky
// factor and inverse of leaves of 129..256 points go to rocSOLVER / rocBLAS on
// the factor path.  The apply runs on this file's kernels only.  Everything is
// FP64.
#include "internal.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace mag {
namespace {

constexpr int SL = 64;      // slab / tile width of every basis
constexpr int KMAXC = 8;    // widest basis: KMAXC * SL columns
constexpr int LMAX = 256;   // largest leaf
constexpr int LSW = 128;    // largest leaf inverted inside LDS (sweep operator)
constexpr int MMAXH = 16;   // largest point dimension
constexpr int ZR = 64;      // rows per sampling workgroup
constexpr int ZC = 16;      // points per sampling column chunk
constexpr int NT = 256;     // threads per workgroup

__device__ inline double sq_acc(double s, double e)
{
#pragma clang fp contract(off)
    double p = e * e;
    return s + p;
}

// SplitMix64 output function (Steele, Lea and Flood, 2014).
__host__ __device__ inline uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Omega (n x ld): N(0, 1) entries (Box-Muller on two hashed uniforms) in the
// first kcols columns, zero in the rest.
__global__ void __launch_bounds__(NT) k_omega(double *__restrict__ Om, int64_t n, int ld, int kcols,
                                              uint64_t seed)
{
    const int64_t total = n * ld;
    for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
        const int c = (int)(e % ld);
        double v = 0.0;
        if (c < kcols) {
            const uint64_t h1 = mix64(seed ^ mix64(2 * (uint64_t)e));
            const uint64_t h2 = mix64(seed ^ mix64(2 * (uint64_t)e + 1));
            const double u1 = (double)((h1 >> 11) + 1) * 0x1.0p-53;  // (0, 1]
            const double u2 = (double)(h2 >> 11) * 0x1.0p-53;        // [0, 1)
            v = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        }
        Om[e] = v;
    }
}

// Sampling product over the sibling pairs of one level, NS 64-column slabs
// (blockIdx.y) of B and out (both n x ld, row-major):
//   out[r, slab] = sum_{c in C} Z(r, c) B[c, slab]   for r in R,
// mode 0: R = left child, C = right child;  mode 1: R = right, C = left.
// bnd: bounds of the children level (2 * tasks + 1 entries).  One workgroup
// per 64-row block of R and NS slabs.  Per chunk of ZC points the Z tile
// (64 x ZC, FP64 exp of exact distances) is formed in LDS by the VALU and
// applied to all NS slabs on the FP64 matrix cores (v_mfma_f64_16x16x4: on
// gfx950 twice the FP64 rate of VALU FMAs, and its operands come one double
// per lane per 16x16x4 step, so LDS traffic stays small): wave w owns the
// 16 NS columns [16 NS w, 16 NS (w + 1)) of the workgroup's output, all 64
// rows, as 4 x NS accumulator blocks of 16 x 16.  The chunk's B rows go
// through registers, loaded while the previous chunk is applied.  Every
// output sums the same chunks in the same order whatever NS is.
typedef double v4d __attribute__((ext_vector_type(4)));

template <int NS, int M>
__global__ void __launch_bounds__(NT)
k_zblock(const double *__restrict__ Xp, int m_rt, double t, const int64_t *__restrict__ bnd, int mode,
         int rbmax, const double *B, double *out, int ld)
{
    // M > 0: compile-time dimension (straight-line distance code); M = 0: m_rt <= MMAXH
    constexpr int MM = (M > 0) ? M : MMAXH;
    const int m = (M > 0) ? M : m_rt;
    constexpr int CC = ZC;       // points per chunk (16)
    constexpr int W = NS * SL;   // output columns of the workgroup
    __shared__ double Bs[CC][W];
    __shared__ double Zs[ZR][CC + 1];
    __shared__ double Xc[MM][CC];
    const int task = blockIdx.x / rbmax, rb = blockIdx.x % rbmax;
    const int col0 = blockIdx.y * W;
    const int64_t a = bnd[2 * task], b = bnd[2 * task + 1], c = bnd[2 * task + 2];
    const int64_t rlo = mode ? b : a, rhi = mode ? c : b;
    const int64_t clo = mode ? a : b, chi = mode ? b : c;
    const int64_t r0 = rlo + (int64_t)rb * ZR;
    if (r0 >= rhi) return;  // uniform per workgroup
    const int nr = (int)min((int64_t)ZR, rhi - r0);
    const int tid = threadIdx.x;
    const int gr = tid & 63, gp = tid >> 6;  // Z-tile generation: row, group of CC / 4 points
    const int lane = tid & 63, wv = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;  // MFMA operand lane roles
    const int cbase = wv * 16 * NS;            // this wave's first output column
    double xr[MM];
#pragma unroll
    for (int l = 0; l < MM; ++l) xr[l] = (l < m && gr < nr) ? Xp[(r0 + gr) * m + l] : 0.0;
    v4d acc[4][NS];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < NS; ++u) acc[i][u] = v4d{0.0, 0.0, 0.0, 0.0};

    // the B rows of a chunk go through registers: the next chunk's are loaded
    // while this one's Z tile is formed and applied
    constexpr int PER = CC * W / NT;
    double breg[PER];
    auto fetch = [&](int64_t cb) {
        const int cn = (int)min((int64_t)CC, chi - cb);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + i * NT;
            const int p = e / W, q = e % W;
            breg[i] = (p < cn) ? B[(cb + p) * ld + col0 + q] : 0.0;
        }
    };
    if (clo < chi) fetch(clo);
    for (int64_t c0 = clo; c0 < chi; c0 += CC) {
        const int cnt = (int)min((int64_t)CC, chi - c0);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + i * NT;
            Bs[e / W][e % W] = breg[i];
        }
        for (int e = tid; e < m * CC; e += NT) {
            const int l = e / CC, p = e % CC;
            Xc[l][p] = (p < cnt) ? Xp[(c0 + p) * m + l] : 0.0;
        }
        __syncthreads();
        if (c0 + CC < chi) fetch(c0 + CC);
        for (int q = 0; q < CC / 4; ++q) {
            const int p = gp * (CC / 4) + q;
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < MM; ++l)
                if (M > 0 || l < m) s = sq_acc(s, xr[l] - Xc[l][p]);
            const double z = zexp(t, s);  // evaluated for padding too, then selected
            Zs[gr][p] = (p < cnt && gr < nr) ? z : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < CC / 4; ++kk) {
            // A(row, k) = Z(16 i + row, 4 kk + k) for row block i: lane (row = li, k = lk)
            double av[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = Zs[16 * i + li][4 * kk + lk];
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                // B(k, j) = Bs(4 kk + k, cbase + 16 u + j): lane (k = lk, j = li)
                const double bv = Bs[4 * kk + lk][cbase + 16 * u + li];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[i][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv, acc[i][u], 0, 0, 0);
            }
        }
    }
    // D(lane, v) = C(lk + 4 v, li) of each 16 x 16 block
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 16 * i + lk + 4 * v;
            if (r < nr) {
#pragma unroll
                for (int u = 0; u < NS; ++u) out[(r0 + r) * ld + col0 + cbase + 16 * u + li] = acc[i][u][v];
            }
        }
}

// Launch k_zblock over `tasks` sibling pairs, `cols` columns (a multiple of 64)
// of B and out: groups of 4 slabs per workgroup, then the remainder in one
// launch of 2 and/or 1 (5 slabs: 4 + 1, so each Z entry is formed twice, not
// five times).  The sums do not depend on the grouping.
void launch_zblock(hipStream_t s, const double *Xp, int m, double t, const int64_t *bnd, int mode, int64_t tasks,
                   int rbmax, const double *B, double *out, int ld, int cols)
{
    const int slabs = cols / SL;
    const unsigned gx = (unsigned)(tasks * rbmax);
    for (int done = 0; done < slabs;) {
        const int rem = slabs - done;
        const int ns = rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
        const dim3 g(gx, (unsigned)(rem / ns));
        const double *Bd = B + done * SL;
        double *od = out + done * SL;
        if (m == 3) {
            if (ns == 4) hipLaunchKernelGGL((k_zblock<4, 3>), g, dim3(NT), 0, s, Xp, m, t, bnd, mode, rbmax, Bd, od, ld);
            else if (ns == 2) hipLaunchKernelGGL((k_zblock<2, 3>), g, dim3(NT), 0, s, Xp, m, t, bnd, mode, rbmax, Bd, od, ld);
            else hipLaunchKernelGGL((k_zblock<1, 3>), g, dim3(NT), 0, s, Xp, m, t, bnd, mode, rbmax, Bd, od, ld);
        } else {
            if (ns == 4) hipLaunchKernelGGL((k_zblock<4, 0>), g, dim3(NT), 0, s, Xp, m, t, bnd, mode, rbmax, Bd, od, ld);
            else if (ns == 2) hipLaunchKernelGGL((k_zblock<2, 0>), g, dim3(NT), 0, s, Xp, m, t, bnd, mode, rbmax, Bd, od, ld);
            else hipLaunchKernelGGL((k_zblock<1, 0>), g, dim3(NT), 0, s, Xp, m, t, bnd, mode, rbmax, Bd, od, ld);
        }
        done += (rem / ns) * ns;
    }
}

// Row range of task i: [bnd[ts*i + to], bnd[ts*i + to + 1]).
__device__ inline void task_range(const int64_t *bnd, int ts, int to, int i, int64_t &lo, int64_t &hi)
{
    lo = bnd[ts * i + to];
    hi = bnd[ts * i + to + 1];
}

// Gram partials A[R]^T B[R] (lda x ldb) per task, per chunk of crows rows,
// per 64 x 64 tile y = (ai, bj) (blockIdx.y):
//   partial[((task * cmax + ch) * ntile + y) * 4096 ..] (tile, row-major).
__global__ void __launch_bounds__(NT)
k_gram_partial(const double *__restrict__ A, int lda, const double *__restrict__ B, int ldb,
               const int64_t *__restrict__ bnd, int ts, int to, int crows, int cmax,
               double *__restrict__ partial)
{
    __shared__ double As[32][SL];
    __shared__ double Bs[32][SL];
    const int task = blockIdx.x / cmax, ch = blockIdx.x % cmax;
    const int nbj = ldb / SL, y = blockIdx.y, ntile = gridDim.y;
    const int ac = (y / nbj) * SL, bc = (y % nbj) * SL;
    int64_t lo, hi;
    task_range(bnd, ts, to, task, lo, hi);
    const int64_t r0 = lo + (int64_t)ch * crows;
    const int64_t r1 = min(hi, r0 + crows);
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int64_t rs = r0; rs < r1; rs += 32) {
        const int cnt = (int)min((int64_t)32, r1 - rs);
        __syncthreads();
        for (int e = tid; e < 32 * SL; e += NT) {
            const int rr = e / SL, q = e % SL;
            As[rr][q] = (rr < cnt) ? A[(rs + rr) * lda + ac + q] : 0.0;
            Bs[rr][q] = (rr < cnt) ? B[(rs + rr) * ldb + bc + q] : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < 32; ++rr) {
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[rr][4 * ty + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[rr][4 * tx + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
    }
    double *o = partial + ((int64_t)(task * cmax + ch) * ntile + y) * (SL * SL);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) o[(4 * ty + i) * SL + 4 * tx + j] = acc[i][j];
}

// Sum of the chunk partials (fixed order) into out[task] = lda x ldb,
// column-major with leading dimension lda.  grid (tasks * ntile, 16)
__global__ void __launch_bounds__(NT)
k_gram_reduce(const double *__restrict__ partial, int cmax, int lda, int ldb, double *__restrict__ out)
{
    const int nbj = ldb / SL, ntile = (lda / SL) * nbj;
    const int task = blockIdx.x / ntile, y = blockIdx.x % ntile;
    const int e = blockIdx.y * NT + threadIdx.x;  // within the tile, row-major
    double s = 0.0;
    for (int ch = 0; ch < cmax; ++ch) s += partial[((int64_t)(task * cmax + ch) * ntile + y) * (SL * SL) + e];
    const int row = (y / nbj) * SL + e / SL, col = (y % nbj) * SL + e % SL;
    out[(int64_t)task * lda * ldb + (int64_t)col * lda + row] = s;
}

// G_task += s I with s = 11 (rows k + k (k + 1)) u tr(G), the shift of
// shifted CholeskyQR (Fukaya, Kannan, Nakatsukasa, Yamamoto and Yanagisawa,
// 2020), so the Cholesky of the Gram matrix of a rank-deficient sample still
// succeeds; an all-zero G becomes the identity.  One workgroup per task.
__global__ void __launch_bounds__(NT)
k_gram_shift(double *__restrict__ G, int k, const int64_t *__restrict__ bnd, int ts, int to)
{
    __shared__ double red[NT];
    double *g = G + (int64_t)blockIdx.x * k * k;
    double tr = 0.0;
    for (int i = threadIdx.x; i < k; i += NT) tr += g[(int64_t)i * k + i];
    red[threadIdx.x] = tr;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    int64_t lo, hi;
    task_range(bnd, ts, to, blockIdx.x, lo, hi);
    const double trace = red[0];
    const double s = (trace > 0.0 && isfinite(trace))
                         ? 11.0 * ((double)(hi - lo) * k + (double)k * (k + 1)) * 0x1.0p-53 * trace
                         : 1.0;
    for (int i = threadIdx.x; i < k; i += NT) g[(int64_t)i * k + i] += s;
}

// Zero the strictly lower triangle of each k x k column-major block (the
// Cholesky leaves it untouched), so the block is R^{-1} for the row products.
__global__ void k_zero_lower(double *__restrict__ R, int k, int64_t count)
{
    const int64_t per = (int64_t)k * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count * per;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t w = e % per;
        const int col = (int)(w / k), row = (int)(w % k);
        if (row > col) R[e] = 0.0;
    }
}

// Row-block products: out[r, slab] = (sub ? out[r, slab] - : ) A[r, :] M[:, slab]
// for the rows r of each task, M = Mb + task * mstride (lda x ldo,
// column-major, leading dimension lda); grid (tasks * rbmax, ldo / 64).
// out must not alias A.
__global__ void __launch_bounds__(NT)
k_rowmul(const double *__restrict__ A, int lda, double *__restrict__ out, int ldo,
         const double *__restrict__ Mb, int64_t mstride, const int64_t *__restrict__ bnd, int ts, int to,
         int rbmax, int sub)
{
    __shared__ double As[64][SL + 1];
    __shared__ double Ms[SL][SL + 1];
    const int task = blockIdx.x / rbmax, rb = blockIdx.x % rbmax;
    const int col0 = blockIdx.y * SL;
    int64_t lo, hi;
    task_range(bnd, ts, to, task, lo, hi);
    const int64_t r0 = lo + (int64_t)rb * 64;
    if (r0 >= hi) return;  // uniform
    const int nr = (int)min((int64_t)64, hi - r0);
    const double *M = Mb + (int64_t)task * mstride;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < lda; k0 += SL) {
        __syncthreads();
        for (int e = tid; e < 64 * SL; e += NT) {
            const int rr = e / SL, q = e % SL;
            As[rr][q] = (rr < nr) ? A[(r0 + rr) * lda + k0 + q] : 0.0;
            // Ms[kk][j] = M(k0 + kk, col0 + j), read down the columns of M
            const int j = e / SL, kk = e % SL;
            Ms[kk][j] = M[(int64_t)(col0 + j) * lda + k0 + kk];
        }
        __syncthreads();
        for (int kk = 0; kk < SL; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[4 * ty + i][kk];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Ms[kk][4 * tx + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 4 * ty + i;
        if (r < nr) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double *p = out + (r0 + r) * ldo + col0 + 4 * tx + j;
                *p = sub ? (*p - acc[i][j]) : acc[i][j];
            }
        }
    }
}

// Copy the rows of the tasks' ranges from src to dst (both n x ld).
__global__ void __launch_bounds__(NT)
k_copy_rows(const double *__restrict__ src, double *__restrict__ dst, int ld, const int64_t *__restrict__ bnd,
            int ts, int to, int rbmax)
{
    const int task = blockIdx.x / rbmax, rb = blockIdx.x % rbmax;
    int64_t lo, hi;
    task_range(bnd, ts, to, task, lo, hi);
    const int64_t r0 = lo + (int64_t)rb * 64;
    const int64_t r1 = min(hi, r0 + 64);
    for (int64_t e = r0 * ld + threadIdx.x; e < r1 * ld; e += NT) dst[e] = src[e];
}

// Inverse of each leaf block Z(leaf, leaf) (exact FP64 entries) by the sweep
// operator (Goodnight, 1979): sweeping every pivot of a symmetric positive
// definite A turns it into -A^{-1}; pivots are the Schur-complement
// diagonals, positive for SPD A.  Leaves of at most LSW points, whole in LDS.
// Dinv: LSW x LSW per leaf (symmetric; the padding is the identity).  A pivot
// that is not positive marks status.
__global__ void __launch_bounds__(NT)
k_leaf_inv(const double *__restrict__ Xp, int m, double t, const int64_t *__restrict__ bndL,
           double *__restrict__ Dinv, int *__restrict__ status)
{
    __shared__ double A[LSW][LSW + 1];
    __shared__ double colk[LSW];
    const int tid = threadIdx.x;
    const int64_t lo = bndL[blockIdx.x], hi = bndL[blockIdx.x + 1];
    const int s = (int)(hi - lo);
    for (int e = tid; e < LSW * LSW; e += NT) {
        const int i = e / LSW, j = e % LSW;
        double v;
        if (i == j) {
            v = 1.0;
        } else if (i < s && j < s) {
            double d2 = 0.0;
            for (int l = 0; l < m; ++l) d2 = sq_acc(d2, Xp[(lo + i) * m + l] - Xp[(lo + j) * m + l]);
            v = zexp(t, d2);
        } else {
            v = 0.0;
        }
        A[i][j] = v;
    }
    bool bad = false;
    for (int k = 0; k < s; ++k) {
        __syncthreads();
        if (tid < LSW) colk[tid] = A[tid][k];
        __syncthreads();
        double akk = colk[k];
        if (!(akk > 0.0) || !isfinite(akk)) {
            bad = true;
            akk = 1.0;
        }
        const double inv = 1.0 / akk;
        for (int e = tid; e < LSW * LSW; e += NT) {
            const int i = e / LSW, j = e % LSW;
            if (i == k && j == k) A[i][j] = -inv;
            else if (i == k) A[i][j] = colk[j] * inv;
            else if (j == k) A[i][j] = colk[i] * inv;
            else A[i][j] -= colk[i] * colk[j] * inv;
        }
    }
    __syncthreads();
    double *D = Dinv + (int64_t)blockIdx.x * LSW * LSW;
    for (int e = tid; e < LSW * LSW; e += NT) {
        const int i = e / LSW, j = e % LSW;
        D[e] = (i < s && j < s) ? -A[i][j] : (i == j ? 1.0 : 0.0);
    }
    if (bad && tid == 0) atomicCAS(&status[kStBreakdown], 0, (int)(lo + 1));
}

// Leaves larger than LSW: the blocks Z(leaf, leaf), padded to ls x ls with the
// identity, written to Dinv for a batched Cholesky factor and inverse in HBM.
// Grid (leaves, chunks); the entries of one leaf are spread over the chunks.
__global__ void __launch_bounds__(NT)
k_leaf_fill(const double *__restrict__ Xp, int m, double t, const int64_t *__restrict__ bndL, int ls,
            double *__restrict__ Dinv)
{
    const int64_t lo = bndL[blockIdx.x], hi = bndL[blockIdx.x + 1];
    const int s = (int)(hi - lo);
    double *D = Dinv + (int64_t)blockIdx.x * ls * ls;
    for (int e = blockIdx.y * NT + threadIdx.x; e < ls * ls; e += gridDim.y * NT) {
        const int i = e / ls, j = e % ls;  // symmetric: row and column order agree
        double v;
        if (i == j) {
            v = 1.0;
        } else if (i < s && j < s) {
            double d2 = 0.0;
            for (int l = 0; l < m; ++l) d2 = sq_acc(d2, Xp[(lo + i) * m + l] - Xp[(lo + j) * m + l]);
            v = zexp(t, d2);
        } else {
            v = 0.0;
        }
        D[e] = v;
    }
}

// A leaf whose batched factorisation reported a failed pivot (info > 0) marks
// status with its first point, as the sweep does.
__global__ void k_leaf_info(const int *__restrict__ info, const int64_t *__restrict__ bndL, int64_t leaves,
                            int *__restrict__ status)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < leaves; i += (int64_t)gridDim.x * blockDim.x)
        if (info[i] != 0) atomicCAS(&status[kStBreakdown], 0, (int)(bndL[i] + 1));
}

// The lower triangle (column-major) of each ls x ls inverse mirrored into its
// upper triangle.
__global__ void __launch_bounds__(NT)
k_leaf_symm(double *__restrict__ Dinv, int ls)
{
    double *D = Dinv + (int64_t)blockIdx.x * ls * ls;
    for (int e = blockIdx.y * NT + threadIdx.x; e < ls * ls; e += gridDim.y * NT) {
        const int c = e / ls, r = e % ls;  // entry (r, c) at D[c ls + r]
        if (r < c) D[e] = D[(int64_t)r * ls + c];
    }
}

// Ph[leaf rows, slab] = Dinv_leaf P[leaf rows, slab] (both n x ld); grid
// (leaves, ld / 64, LS / 128): 128 output rows by 64 columns per workgroup,
// the contraction over the leaf in chunks of 32 through LDS.
template <int LS>
__global__ void __launch_bounds__(NT)
k_leaf_apply(const double *__restrict__ Dinv, const int64_t *__restrict__ bndL, const double *__restrict__ P,
             double *__restrict__ Ph, int ld)
{
    __shared__ double Bs[32][SL];
    __shared__ double Ms[128][33];
    const int64_t lo = bndL[blockIdx.x], hi = bndL[blockIdx.x + 1];
    const int s = (int)(hi - lo);
    const int col0 = blockIdx.y * SL, row0 = blockIdx.z * 128;
    const double *M = Dinv + (int64_t)blockIdx.x * LS * LS;
    const int tid = threadIdx.x;
    const int ty = tid >> 3, tx = tid & 7;  // rows row0 + 4ty.., columns 8tx..
    double acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
    for (int kc = 0; kc < s; kc += 32) {
        __syncthreads();
        for (int e = tid; e < 128 * 32; e += NT) {
            const int i = e / 32, j = e % 32;
            Ms[i][j] = M[(int64_t)(row0 + i) * LS + kc + j];
        }
        for (int e = tid; e < 32 * SL; e += NT) {
            const int rr = e / SL, q = e % SL;
            Bs[rr][q] = (kc + rr < s) ? P[(lo + kc + rr) * ld + col0 + q] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < 32; ++kk) {
            double av[4], bv[8];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = Ms[4 * ty + i][kk];
#pragma unroll
            for (int j = 0; j < 8; ++j) bv[j] = Bs[kk][8 * tx + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = row0 + 4 * ty + i;
        if (r < s) {
#pragma unroll
            for (int j = 0; j < 8; ++j) Ph[(lo + r) * ld + col0 + 8 * tx + j] = acc[i][j];
        }
    }
}

// Per node i (batch of `count`): Bm = G[2i+1], Cm = G[2i] (k x k each, from
// the children's Gram matrices) and S = I, in node storage [Bm | Cm | S].
__global__ void k_node_setup(const double *__restrict__ G, int k, int64_t count, double *__restrict__ W)
{
    const int64_t kk = (int64_t)k * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count * kk;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / kk, w = e % kk;
        double *Wi = W + i * 3 * kk;
        Wi[w] = G[(2 * i + 1) * kk + w];
        Wi[kk + w] = G[(2 * i) * kk + w];
        Wi[2 * kk + w] = (w / k == w % k) ? 1.0 : 0.0;
    }
}

// ---- preconditioner apply ------------------------------------------------------
__global__ void k_gather(const double *__restrict__ r, const int64_t *__restrict__ perm, int64_t n,
                         double *__restrict__ xp)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        xp[i] = r[perm[i]];
}

// z[perm[i]] = xp[i]; z zero on [n, npad)
__global__ void k_scatter(const double *__restrict__ xp, const int64_t *__restrict__ perm, int64_t n,
                          int64_t npad, double *__restrict__ z)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npad; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n) z[perm[i]] = xp[i];
        else z[i] = 0.0;
    }
}

// x[leaf] = Dinv_leaf x[leaf] in place (Dinv symmetric: column access
// coalesces).  A thread per row, the leaf's columns split over NT / LS threads.
template <int LS>
__global__ void __launch_bounds__(NT)
k_leaf_gemv(const double *__restrict__ Dinv, const int64_t *__restrict__ bndL, double *__restrict__ x)
{
    constexpr int SPLIT = NT / LS, KC = LS / SPLIT;
    __shared__ double xs[LS];
    __shared__ double hs[NT];
    const int64_t lo = bndL[blockIdx.x], hi = bndL[blockIdx.x + 1];
    const int s = (int)(hi - lo);
    const int tid = threadIdx.x, row = tid % LS, part = tid / LS;
    if (tid < LS) xs[tid] = (tid < s) ? x[lo + tid] : 0.0;
    __syncthreads();
    const double *D = Dinv + (int64_t)blockIdx.x * LS * LS;
    double acc = 0.0;
    for (int k = part * KC; k < part * KC + KC; ++k) acc = fma(D[k * LS + row], xs[k], acc);
    if (SPLIT == 1) {
        if (row < s) x[lo + row] = acc;
        return;
    }
    hs[tid] = acc;
    __syncthreads();
    if (part == 0 && row < s) {
        double v = acc;
        for (int q = 1; q < SPLIT; ++q) v += hs[q * LS + row];
        x[lo + row] = v;
    }
}

// partial[(c * cmax + ch) * ld + q] = sum_{r in chunk} P[r, q] x[r] over the
// children c, slab blockIdx.y
__global__ void __launch_bounds__(NT)
k_node_dots(const double *__restrict__ P, int ld, const double *__restrict__ x, const int64_t *__restrict__ bnd,
            int crows, int cmax, double *__restrict__ partial)
{
    __shared__ double red[4][SL];
    const int c = blockIdx.x / cmax, ch = blockIdx.x % cmax;
    const int64_t lo = bnd[c], hi = bnd[c + 1];
    const int64_t r0 = lo + (int64_t)ch * crows, r1 = min(hi, r0 + crows);
    const int ql = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int q = blockIdx.y * SL + ql;
    double acc = 0.0;
    for (int64_t r = r0 + g; r < r1; r += 4) acc = fma(P[r * ld + q], x[r], acc);
    red[g][ql] = acc;
    __syncthreads();
    if (g == 0) partial[((int64_t)c * cmax + ch) * ld + q] = ((red[0][ql] + red[1][ql]) + red[2][ql]) + red[3][ql];
}

// Node correction coefficients (one workgroup per node i, k <= 512):
//   s1 = V_J^T x_J, s2 = U_I^T x_I (sums of the dot partials),
//   x1 = S^{-1} (s1 - B s2),  x2 = s2 - C x1,   tv[i] = [x1; x2].
__global__ void __launch_bounds__(NT)
k_node_small(const double *__restrict__ partial, int cmax, int k, const double *__restrict__ W,
             double *__restrict__ tv)
{
    __shared__ double s1[KMAXC * SL], s2[KMAXC * SL], u[KMAXC * SL], x1[KMAXC * SL];
    const int i0 = blockIdx.x, tid = threadIdx.x;
    const int64_t kk = (int64_t)k * k;
    const double *Bm = W + (int64_t)i0 * 3 * kk, *Cm = Bm + kk, *Si = Bm + 2 * kk;
    for (int q = tid; q < k; q += NT) {
        double a = 0.0, b = 0.0;
        for (int ch = 0; ch < cmax; ++ch) {
            a += partial[((int64_t)(2 * i0 + 1) * cmax + ch) * k + q];
            b += partial[((int64_t)(2 * i0) * cmax + ch) * k + q];
        }
        s1[q] = a;
        s2[q] = b;
    }
    __syncthreads();
    for (int r = tid; r < k; r += NT) {  // u = s1 - B s2 (column-major: coalesced over r)
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(Bm[(int64_t)j * k + r], s2[j], acc);
        u[r] = s1[r] - acc;
    }
    __syncthreads();
    for (int r = tid; r < k; r += NT) {  // x1 = S^{-1} u
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(Si[(int64_t)j * k + r], u[j], acc);
        x1[r] = acc;
    }
    __syncthreads();
    double *o = tv + (int64_t)i0 * 2 * k;
    for (int r = tid; r < k; r += NT) {  // x2 = s2 - C x1
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(Cm[(int64_t)j * k + r], x1[j], acc);
        o[r] = x1[r];
        o[k + r] = s2[r] - acc;
    }
}

// x[r] -= Ph[r, :] tv[c/2][(c%2) k ...] for the rows of child c; one
// workgroup per 64-row block, 4 threads per row.
__global__ void __launch_bounds__(NT)
k_node_update(const double *__restrict__ Ph, int k, const int64_t *__restrict__ bnd, int rbmax,
              const double *__restrict__ tv, double *__restrict__ x)
{
    const int c = blockIdx.x / rbmax, rb = blockIdx.x % rbmax;
    const int64_t lo = bnd[c], hi = bnd[c + 1];
    const int64_t r = lo + (int64_t)rb * 64 + (threadIdx.x >> 2);
    const int part = threadIdx.x & 3;
    const int q = k / 4;
    const double *tvec = tv + (int64_t)(c >> 1) * 2 * k + (c & 1) * k + part * q;
    double acc = 0.0;
    if (r < hi) {
        const double *row = Ph + r * k + part * q;
        for (int j = 0; j < q; ++j) acc = fma(row[j], tvec[j], acc);
    }
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    if (r < hi && part == 0) x[r] -= acc;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t boff(int l) { return ((int64_t)1 << l) - 1 + l; }

}  // namespace

// ---- host side -------------------------------------------------------------------

int hodlr_max_leaf() { return LMAX; }
int hodlr_default_leaf() { return LSW; }
int hodlr_max_cols() { return KMAXC * SL; }

// Perfect tree of L levels over n points: level bounds and the permutation
// (recursive coordinate bisection, median of the widest coordinate).
static void build_tree(const std::vector<double> &X, int64_t n, int m, int L, std::vector<int64_t> &perm,
                       std::vector<int64_t> &bnd)
{
    perm.resize(n);
    std::iota(perm.begin(), perm.end(), (int64_t)0);
    bnd.assign(boff(L + 1), 0);
    bnd[boff(0)] = 0;
    bnd[boff(0) + 1] = n;
    for (int l = 0; l < L; ++l) {
        const int64_t nn = (int64_t)1 << l;
        int64_t *b = bnd.data() + boff(l);
        int64_t *c = bnd.data() + boff(l + 1);
        for (int64_t i = 0; i < nn; ++i) {
            const int64_t lo = b[i], hi = b[i + 1], mid = lo + (hi - lo) / 2;
            c[2 * i] = lo;
            c[2 * i + 1] = mid;
            c[2 * i + 2] = hi;
            if (hi - lo < 2) continue;
            int ax = 0;
            double wbest = -1.0;
            for (int a = 0; a < m; ++a) {
                double mn = INFINITY, mx = -INFINITY;
                for (int64_t p = lo; p < hi; ++p) {
                    const double v = X[perm[p] * m + a];
                    mn = std::min(mn, v);
                    mx = std::max(mx, v);
                }
                if (mx - mn > wbest) {
                    wbest = mx - mn;
                    ax = a;
                }
            }
            std::nth_element(perm.begin() + lo, perm.begin() + mid, perm.begin() + hi,
                             [&](int64_t u, int64_t v) {
                                 const double xu = X[u * m + ax], xv = X[v * m + ax];
                                 return xu < xv || (xu == xv && u < v);
                             });
        }
    }
}

int hodlr_levels(int64_t n, int leaf)
{
    int L = 0;
    while (cdiv(n, (int64_t)1 << L) > leaf) ++L;
    return L;
}

// Basis width of level l: rank0 2^{-l/2} + oversample rounded up to a
// multiple of 64, at least 64, at most KMAXC * 64 and at most the smaller
// child (rounded down to 64, but never below 64).
static int level_cols(int l, int rank0, int oversample, int64_t minchild)
{
    const double want = rank0 * std::pow(2.0, -0.5 * l) + oversample;
    int c = (int)std::ceil(want / SL);
    c = std::max(1, std::min(c, KMAXC));
    const int cap = (int)std::max<int64_t>(1, minchild / SL);
    return SL * std::min(c, cap);
}

struct HodlrPlan {
    std::vector<int> k;              // basis width per level
    std::vector<int64_t> poff;       // offset of P_l / Ph_l (doubles)
    std::vector<int64_t> woff;       // offset of level l's node storage (doubles)
    std::vector<int64_t> csz, cmin;  // largest / smallest child of level l's nodes
    std::vector<int> crows, cmax;    // Gram chunking per level
    int64_t ptotal = 0, wtotal = 0, gpart = 0, gout = 0, tbuf = 0, apart = 0, ipiv = 0;
    int kmax = SL;
};

static HodlrPlan make_plan(int64_t n, int L, const std::vector<int64_t> &bnd, int rank0, int oversample)
{
    HodlrPlan pl;
    pl.k.resize(L);
    pl.poff.resize(L + 1);
    pl.woff.resize(L + 1);
    pl.csz.resize(L);
    pl.cmin.resize(L);
    pl.crows.resize(L);
    pl.cmax.resize(L);
    int64_t po = 0, wo = 0;
    for (int l = 0; l < L; ++l) {
        const int64_t nch = (int64_t)2 << l;
        const int64_t *b = bnd.data() + boff(l + 1);
        int64_t mx = 0, mn = INT64_MAX;
        for (int64_t c = 0; c < nch; ++c) {
            mx = std::max(mx, b[c + 1] - b[c]);
            mn = std::min(mn, b[c + 1] - b[c]);
        }
        pl.csz[l] = mx;
        pl.cmin[l] = mn;
        pl.k[l] = level_cols(l, rank0, oversample, mn);
        pl.kmax = std::max(pl.kmax, pl.k[l]);
        // chunks of at least 256 rows, at most 64 chunks per child
        pl.crows[l] = (int)std::max<int64_t>(256, cdiv(cdiv(mx, 64), 32) * 32);
        pl.cmax[l] = (int)cdiv(mx, pl.crows[l]);
        pl.poff[l] = po;
        po += n * pl.k[l];
        pl.woff[l] = wo;
        wo += ((int64_t)1 << l) * 3 * (int64_t)pl.k[l] * pl.k[l];
    }
    pl.poff[L] = po;
    pl.woff[L] = wo;
    pl.ptotal = po;
    pl.wtotal = wo;
    // scratch: Gram partials / results, T, apply partials, pivots
    for (int l = 0; l < L; ++l) {
        const int64_t nch = (int64_t)2 << l;
        for (int lp = 0; lp <= l; ++lp) {
            const int64_t kk = (int64_t)pl.k[l] * pl.k[lp];
            pl.gpart = std::max(pl.gpart, nch * pl.cmax[l] * kk);
            pl.gout = std::max(pl.gout, nch * kk);
            pl.tbuf = std::max(pl.tbuf, (nch / 2) * kk);
        }
        pl.apart = std::max(pl.apart, nch * pl.cmax[l] * (int64_t)pl.k[l]);
        pl.ipiv = std::max(pl.ipiv, (nch / 2) * (int64_t)pl.k[l]);
    }
    return pl;
}

static int blas_handle(mag_ctx *ctx, rocblas_handle &h)
{
    if (!ctx->blas) {
        rocblas_handle nh;
        if (rocblas_create_handle(&nh) != rocblas_status_success) return MAG_EHIP;
        ctx->blas = nh;
    }
    h = (rocblas_handle)ctx->blas;
    return rocblas_set_stream(h, ctx->stream) == rocblas_status_success ? MAG_OK : MAG_EHIP;
}

#define RBCHK(x)                                                                                   \
    do {                                                                                           \
        if ((x) != rocblas_status_success) return MAG_EHIP;                                        \
    } while (0)

int hodlr_factor(mag_ctx *ctx, const double *X, int64_t n, int m, double t, int leaf, int rank0,
                 int oversample, int power, uint64_t seed, HodlrFactor &H)
{
    hipStream_t s = ctx->stream;
    if (m > MMAXH || leaf < 2 || leaf > LMAX || rank0 < 0 || oversample < 0 || power < 0) return MAG_EINVAL;
    const int L = hodlr_levels(n, leaf);
    const int64_t npad = round_up(n, kPad);
    rocblas_handle bh = nullptr;
    if (L > 0 && blas_handle(ctx, bh) != MAG_OK) return MAG_EHIP;

    // tree on the host (coordinates copied once)
    std::vector<double> Xh((size_t)n * m);
    if (hipMemcpyAsync(Xh.data(), X, sizeof(double) * n * m, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MAG_EHIP;
    std::vector<int64_t> perm, bnd;
    build_tree(Xh, n, m, L, perm, bnd);
    int64_t maxleaf = 0;
    for (int64_t i = 0; i < ((int64_t)1 << L); ++i) maxleaf = std::max(maxleaf, bnd[boff(L) + i + 1] - bnd[boff(L) + i]);
    if (maxleaf > LMAX) return MAG_EINTERNAL;
    // leaf storage: LSW x LSW (inverted in LDS) or LMAX x LMAX (batched Cholesky in HBM)
    const int ls = maxleaf <= LSW ? LSW : LMAX;
    std::vector<double> Xp((size_t)n * m);
    for (int64_t i = 0; i < n; ++i)
        for (int l = 0; l < m; ++l) Xp[i * m + l] = Xh[perm[i] * m + l];
    const HodlrPlan pl = make_plan(n, L, bnd, rank0, oversample);

    // device workspace
    const int64_t leaves = (int64_t)1 << L;
    const size_t nd = (size_t)n * m + 2 * (size_t)pl.ptotal + 2 * (size_t)n * pl.kmax +
                      (size_t)leaves * ls * ls + (size_t)pl.wtotal + (size_t)pl.gpart + 2 * (size_t)pl.gout +
                      (size_t)pl.tbuf + (size_t)pl.apart + (size_t)leaves * 2 * pl.kmax + 2 * (size_t)npad + 64;
    const size_t nint = (size_t)n + bnd.size() + 16;
    const size_t nsmall = (size_t)pl.ipiv + leaves + 64;  // rocsolver pivots and infos (int32)
    if (ensure(ctx, ctx->hodlr, sizeof(double) * nd + sizeof(int64_t) * nint + sizeof(int) * nsmall + 1024) !=
        MAG_OK)
        return MAG_ENOMEM;
    double *p = (double *)ctx->hodlr.p;
    H.Xp = p; p += (size_t)n * m;
    H.P = p; p += pl.ptotal;
    H.Ph = p; p += pl.ptotal;
    double *Om = p; p += (size_t)n * pl.kmax;
    double *W2 = p; p += (size_t)n * pl.kmax;
    H.Dinv = p; p += (size_t)leaves * ls * ls;
    H.W = p; p += pl.wtotal;
    double *gpart = p; p += pl.gpart;
    double *G = p; p += pl.gout;
    double *G2 = p; p += pl.gout;
    double *T = p; p += pl.tbuf;
    H.apart = p; p += pl.apart;
    H.tv = p; p += (size_t)leaves * 2 * pl.kmax;
    H.xp = p; p += (size_t)2 * npad;
    p += 64;
    int64_t *ip = (int64_t *)p;
    H.perm = ip; ip += n;
    H.bnd = ip; ip += bnd.size();
    int *ipiv = (int *)(ip + 8);
    int *rinfo = ipiv + pl.ipiv;
    H.n = n;
    H.m = m;
    H.t = t;
    H.L = L;
    H.ls = ls;
    H.npad = npad;
    H.bnd_host = bnd;
    H.k = pl.k;
    H.poff = pl.poff;
    H.woff = pl.woff;
    H.crows = pl.crows;
    H.cmax = pl.cmax;
    H.csz = pl.csz;
    int *status = (int *)ctx->ints.p;  // status words at the start of the int block

    if (hipMemcpyAsync(H.Xp, Xp.data(), sizeof(double) * n * m, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(H.perm, perm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(H.bnd, bnd.data(), sizeof(int64_t) * bnd.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return MAG_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MAG_EHIP;  // the host vectors must outlive the copies
    launch_fill_ints(s, status, 8, 0);

    auto gram = [&](const double *A, int lda, const double *B, int ldb, const int64_t *b, int ts, int to,
                    int64_t tasks, int l, double *out) {
        const int nt = (lda / SL) * (ldb / SL);
        hipLaunchKernelGGL(k_gram_partial, dim3((unsigned)(tasks * pl.cmax[l]), (unsigned)nt), dim3(NT), 0, s, A,
                           lda, B, ldb, b, ts, to, pl.crows[l], pl.cmax[l], gpart);
        hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)(tasks * nt), SL * SL / NT), dim3(NT), 0, s, gpart,
                           pl.cmax[l], lda, ldb, out);
    };
    const double one = 1.0, mone = -1.0, zero = 0.0;

    // 1. bases of every level: sample, orthonormalise (shifted CholeskyQR, three
    // passes), optionally iterate the subspace, project
    for (int l = 0; l < L; ++l) {
        const int k = pl.k[l];
        const int64_t tasks = (int64_t)1 << l;
        const int64_t *bch = H.bnd + boff(l + 1);
        const int rb = (int)cdiv(pl.csz[l], 64);
        double *Pl = H.P + pl.poff[l];
        hipLaunchKernelGGL(k_omega, dim3(2048), dim3(NT), 0, s, Om, n, k, k,
                           mix64(seed + 0x51ed2701ull * (uint64_t)(l + 1)));
        launch_zblock(s, H.Xp, m, t, bch, 0, tasks, rb, Om, Pl, k, k);
        double *src = Pl, *dst = W2;
        // orthonormalise the rows of the left (side 0) or right (side 1)
        // children of src; the result ends in src (the buffers swap)
        auto orth = [&](int side) -> int {
            for (int pass = 0; pass < 3; ++pass) {
                gram(src, k, src, k, bch, 2, side, tasks, l, G);
                hipLaunchKernelGGL(k_gram_shift, dim3((unsigned)tasks), dim3(NT), 0, s, G, k, bch, 2, side);
                RBCHK(rocsolver_dpotrf_strided_batched(bh, rocblas_fill_upper, k, G, k, (rocblas_stride)k * k,
                                                       rinfo, (rocblas_int)tasks));
                RBCHK(rocsolver_dtrtri_strided_batched(bh, rocblas_fill_upper, rocblas_diagonal_non_unit, k, G, k,
                                                       (rocblas_stride)k * k, rinfo, (rocblas_int)tasks));
                hipLaunchKernelGGL(k_zero_lower, dim3(1024), dim3(NT), 0, s, G, k, tasks);
                hipLaunchKernelGGL(k_rowmul, dim3((unsigned)(tasks * rb), (unsigned)(k / SL)), dim3(NT), 0, s, src,
                                   k, dst, k, G, (int64_t)k * k, bch, 2, side, rb, 0);
                std::swap(src, dst);
            }
            return MAG_OK;
        };
        if (orth(0) != MAG_OK) return MAG_EHIP;
        for (int q = 0; q < power; ++q) {
            // subspace iteration with an orthonormalisation after every product:
            // Q_J = orth(Z(J, I) Q_I), then Q_I = orth(Z(I, J) Q_J).  Each product
            // reads one side's rows of src and writes the other side's (in place);
            // the side an orthonormalisation leaves behind in the other buffer is
            // the one the next product overwrites.
            launch_zblock(s, H.Xp, m, t, bch, 1, tasks, rb, src, src, k, k);
            if (orth(1) != MAG_OK) return MAG_EHIP;
            launch_zblock(s, H.Xp, m, t, bch, 0, tasks, rb, src, src, k, k);
            if (orth(0) != MAG_OK) return MAG_EHIP;
        }
        // the basis of the left children into P_l (an odd number of passes ends in W2)
        if (src != Pl)
            hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)(tasks * rb)), dim3(NT), 0, s, src, Pl, k, bch, 2, 0,
                               rb);
        launch_zblock(s, H.Xp, m, t, bch, 1, tasks, rb, Pl, Pl, k, k);
    }

    // 2. leaves: exact inverses, applied to every level's basis
    const int64_t *bL = H.bnd + boff(L);
    if (ls == LSW) {
        hipLaunchKernelGGL(k_leaf_inv, dim3((unsigned)leaves), dim3(NT), 0, s, H.Xp, m, t, bL, H.Dinv, status);
    } else {
        // Cholesky factor and inverse of the padded blocks, batched in HBM (lower, column-major)
        if (!bh && blas_handle(ctx, bh) != MAG_OK) return MAG_EHIP;
        const unsigned chunks = (unsigned)(ls * ls / (NT * 16));
        hipLaunchKernelGGL(k_leaf_fill, dim3((unsigned)leaves, chunks), dim3(NT), 0, s, H.Xp, m, t, bL, ls, H.Dinv);
        RBCHK(rocsolver_dpotrf_strided_batched(bh, rocblas_fill_lower, ls, H.Dinv, ls, (rocblas_stride)ls * ls, rinfo,
                                               (rocblas_int)leaves));
        hipLaunchKernelGGL(k_leaf_info, dim3((unsigned)cdiv(leaves, NT)), dim3(NT), 0, s, rinfo, bL, leaves, status);
        RBCHK(rocsolver_dpotri_strided_batched(bh, rocblas_fill_lower, ls, H.Dinv, ls, (rocblas_stride)ls * ls, rinfo,
                                               (rocblas_int)leaves));
        hipLaunchKernelGGL(k_leaf_info, dim3((unsigned)cdiv(leaves, NT)), dim3(NT), 0, s, rinfo, bL, leaves, status);
        hipLaunchKernelGGL(k_leaf_symm, dim3((unsigned)leaves, chunks), dim3(NT), 0, s, H.Dinv, ls);
    }
    for (int l = 0; l < L; ++l) {
        const dim3 g((unsigned)leaves, (unsigned)(pl.k[l] / SL), (unsigned)(ls / 128));
        if (ls == LSW)
            hipLaunchKernelGGL(k_leaf_apply<LSW>, g, dim3(NT), 0, s, H.Dinv, bL, H.P + pl.poff[l],
                               H.Ph + pl.poff[l], pl.k[l]);
        else
            hipLaunchKernelGGL(k_leaf_apply<LMAX>, g, dim3(NT), 0, s, H.Dinv, bL, H.P + pl.poff[l],
                               H.Ph + pl.poff[l], pl.k[l]);
    }

    // 3. bottom-up Woodbury factors
    for (int l = L - 1; l >= 0; --l) {
        const int k = pl.k[l];
        const int64_t kk = (int64_t)k * k;
        const int64_t tasks = (int64_t)1 << l, nch = 2 * tasks;
        const int64_t *bch = H.bnd + boff(l + 1);
        const int rb = (int)cdiv(pl.csz[l], 64);
        double *Pl = H.P + pl.poff[l];
        double *Phl = H.Ph + pl.poff[l];
        double *Wl = H.W + pl.woff[l];
        // B = V_J^T H_J^{-1} V_J, C = U_I^T H_I^{-1} U_I;  S = I - B C;  S^{-1} by LU
        gram(Pl, k, Phl, k, bch, 1, 0, nch, l, G);
        hipLaunchKernelGGL(k_node_setup, dim3(1024), dim3(NT), 0, s, G, k, tasks, Wl);
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_none, rocblas_operation_none, k, k, k, &mone, Wl, k,
                                            3 * kk, Wl + kk, k, 3 * kk, &one, Wl + 2 * kk, k, 3 * kk,
                                            (rocblas_int)tasks));
        RBCHK(rocsolver_dgetrf_strided_batched(bh, k, k, Wl + 2 * kk, k, 3 * kk, ipiv, k, rinfo, (rocblas_int)tasks));
        RBCHK(rocsolver_dgetri_strided_batched(bh, k, Wl + 2 * kk, k, 3 * kk, ipiv, k, rinfo, (rocblas_int)tasks));
        // corrections of the coarser levels' bases: for each l' < l, with
        // S_c = P_l[c]^T Ph_l'[c]:  X1 = S^{-1} (S_J - B S_I),  X2 = S_I - C X1,
        //   Ph_l'[I] -= Ph_l[I] X1,   Ph_l'[J] -= Ph_l[J] X2
        for (int lp = 0; lp < l; ++lp) {
            const int kp = pl.k[lp];
            const int64_t kkp = (int64_t)k * kp;
            double *Phlp = H.Ph + pl.poff[lp];
            gram(Pl, k, Phlp, kp, bch, 1, 0, nch, l, G2);
            // G2[2i+1] := S_J - B S_I (in place)
            RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_none, rocblas_operation_none, k, kp, k, &mone,
                                                Wl, k, 3 * kk, G2, k, 2 * kkp, &one, G2 + kkp, k, 2 * kkp,
                                                (rocblas_int)tasks));
            // T[i] := S^{-1} G2[2i+1]
            RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_none, rocblas_operation_none, k, kp, k, &one,
                                                Wl + 2 * kk, k, 3 * kk, G2 + kkp, k, 2 * kkp, &zero, T, k, kkp,
                                                (rocblas_int)tasks));
            // G2[2i] := S_I - C T[i]
            RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_none, rocblas_operation_none, k, kp, k, &mone,
                                                Wl + kk, k, 3 * kk, T, k, kkp, &one, G2, k, 2 * kkp,
                                                (rocblas_int)tasks));
            hipLaunchKernelGGL(k_rowmul, dim3((unsigned)(tasks * rb), (unsigned)(kp / SL)), dim3(NT), 0, s, Phl, k,
                               Phlp, kp, T, kkp, bch, 2, 0, rb, 1);
            hipLaunchKernelGGL(k_rowmul, dim3((unsigned)(tasks * rb), (unsigned)(kp / SL)), dim3(NT), 0, s, Phl, k,
                               Phlp, kp, G2, 2 * kkp, bch, 2, 1, rb, 1);
        }
    }
    if (hipGetLastError() != hipSuccess) return MAG_EHIP;
    int st[8];
    if (hipMemcpyAsync(st, status, sizeof(st), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MAG_EHIP;
    if (st[kStBreakdown] > 0) return MAG_ENOTPD;  // a leaf block is not positive definite
    return MAG_OK;
}

// z = H^{-1} r (r, z: npad vectors in the caller's point order; z zero in the padding)
void hodlr_apply(hipStream_t s, const HodlrFactor &H, const double *r, double *z)
{
    const int64_t n = H.n;
    const int L = H.L;
    const int64_t leaves = (int64_t)1 << L;
    const unsigned gb = (unsigned)std::min<int64_t>(cdiv(H.npad, 256), 2048);
    hipLaunchKernelGGL(k_gather, dim3(gb), dim3(256), 0, s, r, H.perm, n, H.xp);
    if (H.ls == LSW)
        hipLaunchKernelGGL(k_leaf_gemv<LSW>, dim3((unsigned)leaves), dim3(NT), 0, s, H.Dinv, H.bnd + boff(L), H.xp);
    else
        hipLaunchKernelGGL(k_leaf_gemv<LMAX>, dim3((unsigned)leaves), dim3(NT), 0, s, H.Dinv, H.bnd + boff(L), H.xp);
    for (int l = L - 1; l >= 0; --l) {
        const int k = H.k[l];
        const int64_t tasks = (int64_t)1 << l, nch = 2 * tasks;
        const int rb = (int)cdiv(H.csz[l], 64);
        const int64_t *bch = H.bnd + boff(l + 1);
        hipLaunchKernelGGL(k_node_dots, dim3((unsigned)(nch * H.cmax[l]), (unsigned)(k / SL)), dim3(NT), 0, s,
                           H.P + H.poff[l], k, H.xp, bch, H.crows[l], H.cmax[l], H.apart);
        hipLaunchKernelGGL(k_node_small, dim3((unsigned)tasks), dim3(NT), 0, s, H.apart, H.cmax[l], k,
                           H.W + H.woff[l], H.tv);
        hipLaunchKernelGGL(k_node_update, dim3((unsigned)(nch * rb)), dim3(NT), 0, s, H.Ph + H.poff[l], k, bch, rb,
                           H.tv, H.xp);
    }
    hipLaunchKernelGGL(k_scatter, dim3(gb), dim3(256), 0, s, H.xp, H.perm, n, H.npad, z);
}


// ==== HSS with nested bases and its ULV factorisation ==========================
// The hierarchically semiseparable form behind Section 3.2's solver: on the
// same cluster tree, every node tau below the root has a basis U_tau of the
// off-diagonal block row Z(I_tau, rest), nested: U_tau = diag(U_a, U_b) R_tau
// for its children a, b (so only the leaves' bases and the small R_tau are
// stored), and sibling blocks are Z(I_a, I_b) ~ U_a B_ab U_b^T.
//
// Construction (randomized, projected samples).  S = (Z - leaf blocks) Omega for
// one Gaussian Omega (n x r), summed from the sibling-pair products of every
// level.  A leaf's basis spans the leading eigenvectors of T T^T, T = S(leaf);
// with S~ = U^T T and O~ = U^T Omega(leaf) kept per node, a parent's sample of
// its own off-diagonal block row, in its children's basis coordinates, is
//   T_tau = [S~_a - B_ab O~_b ; S~_b - B_ab^T O~_a]
// (the sibling block is removed), and R_tau spans the leading eigenvectors of
// T_tau T_tau^T.  B_ab = U_a^T Z(I_a, I_b) U_b with the explicit bases.  The
// full eigenvector matrix Q_tau = [Q_e | R_tau] (ascending eigenvalues) is kept:
// it is the orthogonal transform of the ULV step.
//
// ULV (bottom-up).  A node's block D (the leaf block of Z, or the children's
// Schur complements coupled by B) becomes Q^T D Q; the first e = a - k
// unknowns touch nothing outside the node, so they are eliminated by a
// Cholesky factor L_e, and the Schur complement of the k basis unknowns
// D_ss - W W^T (W = D_se L_e^{-T}) is passed to the parent.  The root's block
// is factored whole.  The apply runs the same steps on a vector: up the tree
// b~ = Q^T b, y_e = L_e^{-1} b~_e, b^ = b~_s - W y_e; the root solve; down the
// tree x_e = L_e^{-T} (y_e - W^T x_s), x = Q [x_e; x_s].
namespace {

// T[leaf] (ell x r, column-major) = S(rows of the leaf, :) (S: n x r row-major); zero padding rows.
__global__ void k_hss_gather_rows(const double *__restrict__ S, int r, const int64_t *__restrict__ bndL, int ell,
                                  int64_t leaves, double *__restrict__ T)
{
    const int64_t blk = (int64_t)ell * r, total = leaves * blk;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t leaf = e / blk, w = e % blk;
        const int j = (int)(w / ell), i = (int)(w % ell);
        const int64_t lo = bndL[leaf], hi = bndL[leaf + 1];
        T[e] = (lo + i < hi) ? S[(lo + i) * r + j] : 0.0;
    }
}

// U (n x k, row-major) from the last k columns of each leaf's Q (ell x ell).
__global__ void k_hss_scatter_basis(const double *__restrict__ Q, int ell, int k, const int64_t *__restrict__ bndL,
                                    int64_t leaves, double *__restrict__ U)
{
    const int64_t blk = (int64_t)ell * k, total = leaves * blk;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t leaf = e / blk, w = e % blk;
        const int i = (int)(w / k), c = (int)(w % k);
        const int64_t lo = bndL[leaf], hi = bndL[leaf + 1];
        if (lo + i < hi) U[(lo + i) * k + c] = Q[leaf * (int64_t)ell * ell + (int64_t)(ell - k + c) * ell + i];
    }
}

// Rs[2p + h] (kc x k, column-major) = rows h kc .. of the last k columns of
// Q[p] (a x a): the blocks R_c of the nested basis, for the row products.
__global__ void k_hss_split_R(const double *__restrict__ Q, int a, int k, int kc, int64_t parents,
                              double *__restrict__ Rs)
{
    const int64_t blk = (int64_t)kc * k, total = 2 * parents * blk;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ch = e / blk, w = e % blk;
        const int c = (int)(w / kc), i = (int)(w % kc);
        const int64_t p = ch / 2, h = ch % 2;
        Rs[e] = Q[p * (int64_t)a * a + (int64_t)(a - k + c) * a + h * kc + i];
    }
}

// dst[p] (2 kc x cols, column-major) = [child 2p; child 2p+1], child c's block
// at src + c * sstride + soff with leading dimension lds.
__global__ void k_hss_stack(const double *__restrict__ src, int64_t sstride, int lds, int soff, int kc, int cols,
                            int64_t parents, double *__restrict__ dst)
{
    const int a = 2 * kc;
    const int64_t blk = (int64_t)a * cols, total = parents * blk;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / blk, w = e % blk;
        const int j = (int)(w / a), i = (int)(w % a);
        const int h = i >= kc ? 1 : 0;
        dst[e] = src[(2 * p + h) * sstride + (int64_t)j * lds + soff + (i - h * kc)];
    }
}

// D[leaf] (ell x ell, column-major): Z on the leaf's points (FP64, the entry of
// the matrix-free product), identity on the padding.
__global__ void k_hss_leaf_block(const double *__restrict__ Xp, int m, double t, const int64_t *__restrict__ bndL,
                                 int ell, int64_t leaves, double *__restrict__ D)
{
    const int64_t blk = (int64_t)ell * ell, total = leaves * blk;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t leaf = e / blk, w = e % blk;
        const int j = (int)(w / ell), i = (int)(w % ell);
        const int64_t lo = bndL[leaf];
        const int sz = (int)(bndL[leaf + 1] - lo);
        double v;
        if (i == j) {
            v = 1.0;
        } else if (i < sz && j < sz) {
            double q = 0.0;
            for (int l = 0; l < m; ++l) q = sq_acc(q, Xp[(lo + i) * m + l] - Xp[(lo + j) * m + l]);
            v = zexp(t, q);
        } else {
            v = 0.0;
        }
        D[e] = v;
    }
}

// D[p] (2 kc x 2 kc) = [[S_a, B], [B^T, S_b]] with S_c the trailing kc x kc
// block (rows and columns e .. e + kc) of child c's Dt (ac x ac) and B = Bc[p]
// (kc x kc, column-major).
__global__ void k_hss_assemble(const double *__restrict__ Dtc, int ac, int kc, const double *__restrict__ Bc,
                               int64_t parents, double *__restrict__ D)
{
    const int a = 2 * kc, ec = ac - kc;
    const int64_t blk = (int64_t)a * a, total = parents * blk;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / blk, w = e % blk;
        const int j = (int)(w / a), i = (int)(w % a);
        const int hi = i >= kc ? 1 : 0, hj = j >= kc ? 1 : 0;
        const int ii = i - hi * kc, jj = j - hj * kc;
        double v;
        if (hi == hj) v = Dtc[(2 * p + hi) * (int64_t)ac * ac + (int64_t)(ec + jj) * ac + (ec + ii)];
        else if (hj) v = Bc[p * (int64_t)kc * kc + (int64_t)jj * kc + ii];
        else v = Bc[p * (int64_t)kc * kc + (int64_t)ii * kc + jj];
        D[e] = v;
    }
}

// xl[leaf] (ell) = r at the leaf's points (tree order through perm), zero padding.
__global__ void k_hss_gather_vec(const double *__restrict__ r, const int64_t *__restrict__ perm,
                                 const int64_t *__restrict__ bndL, int ell, int64_t leaves, double *__restrict__ xl)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < leaves * ell; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t leaf = e / ell;
        const int i = (int)(e % ell);
        const int64_t lo = bndL[leaf], hi = bndL[leaf + 1];
        xl[e] = (lo + i < hi) ? r[perm[lo + i]] : 0.0;
    }
}

// z[perm[p]] = x at tree position p (leaf-padded layout), zero on [n, npad).
__global__ void k_hss_scatter_vec(const double *__restrict__ xl, const int64_t *__restrict__ perm,
                                  const int64_t *__restrict__ bndL, int ell, int64_t leaves, int64_t n, int64_t npad,
                                  double *__restrict__ z)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < leaves * ell; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t leaf = e / ell;
        const int i = (int)(e % ell);
        const int64_t lo = bndL[leaf], hi = bndL[leaf + 1];
        if (lo + i < hi) z[perm[lo + i]] = xl[e];
    }
    for (int64_t e = n + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npad; e += (int64_t)gridDim.x * blockDim.x)
        z[e] = 0.0;
}

// v[tau] (a) = [ub[tau][0 .. e); x of the parent, half tau % 2 (k entries)].
__global__ void k_hss_down_vec(const double *__restrict__ ub, const double *__restrict__ xpar, int apar, int a, int k,
                               int64_t count, double *__restrict__ v)
{
    const int e0 = a - k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count * a; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tau = e / a;
        const int i = (int)(e % a);
        v[e] = (i < e0) ? ub[e] : xpar[(tau / 2) * apar + (tau % 2) * k + (i - e0)];
    }
}

// ---- batched dense matrix-vector products of the HSS apply ------------------
// One problem per node: A column-major (ld lda, node stride sA), x and y with
// node strides sx and sy.  Every sum runs in a fixed order, so the apply is
// bitwise reproducible.

__device__ inline double hss_wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Transposed: y[j] = beta y[j] + alpha sum_i A[i + j lda] x[i] for j < N, i over
// [0, M) or, lower, [j, M).  One wave per output (column j is contiguous).
__global__ void __launch_bounds__(NT)
k_bgemv_t(const double *__restrict__ A, int lda, int64_t sA, const double *__restrict__ x, int64_t sx,
          double *__restrict__ y, int64_t sy, int M, int N, double alpha, double beta, int lower)
{
    const int node = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = blockIdx.x * (NT / 64) + wv;
    if (j >= N) return;  // whole waves; no barriers below
    const double *Aj = A + node * sA + (int64_t)j * lda;
    const double *xn = x + node * sx;
    double acc = 0.0;
    for (int i = (lower ? j : 0) + lane; i < M; i += 64) acc = fma(Aj[i], xn[i], acc);
    acc = hss_wave_sum(acc);
    if (lane == 0) {
        double *yn = y + node * sy;
        yn[j] = (beta == 0.0 ? 0.0 : beta * yn[j]) + alpha * acc;
    }
}

// Not transposed: y[i] = beta y[i] + alpha sum_j A[i + j lda] x[j] for i < M, j
// over [0, N) or, lower, [0, min(i + 1, N)).  One thread per row; the columns
// split into gridDim.y chunks of cs, whose partial sums go to part (node, split,
// row) for k_bgemv_n_reduce when there is more than one.
__global__ void __launch_bounds__(NT)
k_bgemv_n(const double *__restrict__ A, int lda, int64_t sA, const double *__restrict__ x, int64_t sx,
          double *__restrict__ y, int64_t sy, double *__restrict__ part, int M, int N, int cs, double alpha,
          double beta, int lower)
{
    __shared__ double xs[NT];
    const int node = blockIdx.z, sp = blockIdx.y, S = gridDim.y;
    const int i = blockIdx.x * NT + threadIdx.x;
    const int c0 = sp * cs, c1 = min(N, c0 + cs);
    const double *An = A + node * sA;
    const double *xn = x + node * sx;
    double acc = 0.0;
    for (int jb = c0; jb < c1; jb += NT) {
        const int cnt = min(NT, c1 - jb);
        __syncthreads();
        if (threadIdx.x < cnt) xs[threadIdx.x] = xn[jb + threadIdx.x];
        __syncthreads();
        if (i < M) {
            const int jend = lower ? min(cnt, i - jb + 1) : cnt;
            for (int q = 0; q < jend; ++q) acc = fma(An[i + (int64_t)(jb + q) * lda], xs[q], acc);
        }
    }
    if (i < M) {
        if (S == 1) {
            double *yn = y + node * sy;
            yn[i] = (beta == 0.0 ? 0.0 : beta * yn[i]) + alpha * acc;
        } else {
            part[((int64_t)node * S + sp) * M + i] = acc;
        }
    }
}

__global__ void __launch_bounds__(NT)
k_bgemv_n_reduce(const double *__restrict__ part, double *__restrict__ y, int64_t sy, int M, int S, int64_t nodes,
                 double alpha, double beta)
{
    for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < nodes * M; e += (int64_t)gridDim.x * NT) {
        const int64_t node = e / M;
        const int i = (int)(e % M);
        double s = 0.0;
        for (int q = 0; q < S; ++q) s += part[(node * S + q) * M + i];
        double *yn = y + node * sy;
        yn[i] = (beta == 0.0 ? 0.0 : beta * yn[i]) + alpha * s;
    }
}

// y[node][0, e) = x[node][0, e), node strides a
__global__ void k_hss_copy_head(const double *__restrict__ x, double *__restrict__ y, int a, int e, int64_t nodes)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nodes * e; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t node = q / e;
        const int i = (int)(q % e);
        y[node * a + i] = x[node * a + i];
    }
}

// D[node][i][i] += sigma for i < e (the block to eliminate), every node.
__global__ void k_hss_shift(double *__restrict__ D, int a, int e, int64_t nodes, double sigma)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nodes * e; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t node = q / e;
        const int i = (int)(q % e);
        D[node * (int64_t)a * a + (int64_t)i * a + i] += sigma;
    }
}

// largest |entry| of the diagonal of each node's first e x e block, into out[0]
__global__ void k_hss_diagmax(const double *__restrict__ D, int a, int e, int64_t nodes, double *__restrict__ out)
{
    __shared__ double red[NT];
    double v = 0.0;
    for (int64_t q = threadIdx.x; q < nodes * e; q += NT) {
        const int64_t node = q / e;
        const int i = (int)(q % e);
        v = fmax(v, fabs(D[node * (int64_t)a * a + (int64_t)i * a + i]));
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

inline unsigned hss_grid(int64_t total)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + NT - 1) / NT, 4096));
}

// Capacity of the apply's partial-sum buffer (doubles).
constexpr int64_t kHssPart = (int64_t)1 << 19;

void launch_bgemv_t(hipStream_t s, const double *A, int lda, int64_t sA, const double *x, int64_t sx, double *y,
                    int64_t sy, int M, int N, int64_t nodes, double alpha, double beta, bool lower)
{
    if (N <= 0 || nodes <= 0) return;
    const dim3 g((unsigned)((N + NT / 64 - 1) / (NT / 64)), (unsigned)nodes);
    hipLaunchKernelGGL(k_bgemv_t, g, dim3(NT), 0, s, A, lda, sA, x, sx, y, sy, M, N, alpha, beta, lower ? 1 : 0);
}

void launch_bgemv_n(hipStream_t s, const double *A, int lda, int64_t sA, const double *x, int64_t sx, double *y,
                    int64_t sy, double *part, int M, int N, int64_t nodes, double alpha, double beta, bool lower)
{
    if (M <= 0 || nodes <= 0) return;
    const int64_t rb = (M + NT - 1) / NT;
    // column splits until about 1024 workgroups, within the partial buffer
    int64_t S = std::max<int64_t>(1, std::min<int64_t>((1024 + rb * nodes - 1) / (rb * nodes), (N + 63) / 64));
    while (S > 1 && nodes * S * M > kHssPart) --S;
    int cs = (int)((N + S - 1) / S);
    cs = (cs + 63) / 64 * 64;
    S = std::max<int64_t>(1, (N + cs - 1) / cs);
    const dim3 g((unsigned)rb, (unsigned)S, (unsigned)nodes);
    hipLaunchKernelGGL(k_bgemv_n, g, dim3(NT), 0, s, A, lda, sA, x, sx, y, sy, part, M, N, cs, alpha, beta,
                       lower ? 1 : 0);
    if (S > 1)
        hipLaunchKernelGGL(k_bgemv_n_reduce, dim3(hss_grid(nodes * M)), dim3(NT), 0, s, part, y, sy, M, (int)S, nodes,
                           alpha, beta);
}

}  // namespace

#define HSSCHK(x)                                                                                  \
    do {                                                                                           \
        const int rc_ = (x);                                                                       \
        if (rc_ != MAG_OK) return rc_;                                                             \
    } while (0)

int hss_factor(mag_ctx *ctx, const double *X, int64_t n, int m, double t, int leaf, int rank0, int oversample,
               uint64_t seed, HssFactor &H)
{
    hipStream_t s = ctx->stream;
    if (m > MMAXH || leaf < 2 || leaf > LMAX || rank0 < 0 || oversample < 0 || n < 2) return MAG_EINVAL;
    const int L = hodlr_levels(n, leaf);
    const int64_t npad = round_up(n, kPad);
    rocblas_handle bh = nullptr;
    if (blas_handle(ctx, bh) != MAG_OK) return MAG_EHIP;

    std::vector<double> Xh((size_t)n * m);
    if (hipMemcpyAsync(Xh.data(), X, sizeof(double) * n * m, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MAG_EHIP;
    std::vector<int64_t> perm, bnd;
    build_tree(Xh, n, m, L, perm, bnd);
    const int64_t leaves = (int64_t)1 << L;
    int64_t minleaf = INT64_MAX, maxleaf = 0;
    for (int64_t i = 0; i < leaves; ++i) {
        const int64_t sz = bnd[boff(L) + i + 1] - bnd[boff(L) + i];
        minleaf = std::min(minleaf, sz);
        maxleaf = std::max(maxleaf, sz);
    }
    if (maxleaf > LMAX || minleaf < 1) return MAG_EINTERNAL;
    // bases are stored in 64-column slabs: every leaf needs at least 64 points
    if (L > 0 && minleaf < SL) return MAG_EINVAL;
    std::vector<double> Xp((size_t)n * m);
    for (int64_t i = 0; i < n; ++i)
        for (int l = 0; l < m; ++l) Xp[i * m + l] = Xh[perm[i] * m + l];

    // ranks: level l >= 1 keeps k[l] columns, a multiple of 64 within [64, 512]
    // from 8 rank0 2^{-l/2} + oversample, at most its active size a[l] (at the
    // leaves, the smallest leaf, so no basis vector lives on padding).  A node's
    // basis covers its whole off-diagonal block row (the near field on every
    // side), not one sibling block as in the HODLR, hence the factor 8: on the
    // noisy torus at n = 131072 the factor 1 schedule needed diagonal shifts and
    // 400 GMRES iterations, the factor 8 one none and 80-95.
    const int ell = (int)maxleaf;
    std::vector<int> k(L + 1, 0), a(L + 1, 0);
    auto cap = [&](int l) {
        const double want = 8.0 * rank0 * std::pow(2.0, -0.5 * l) + oversample;
        return SL * std::max(1, std::min((int)std::ceil(want / SL), KMAXC));
    };
    if (L == 0) {
        a[0] = ell;
    } else {
        a[L] = ell;
        k[L] = std::min<int>(cap(L), (int)(minleaf / SL) * SL);
        for (int l = L - 1; l >= 1; --l) {
            a[l] = 2 * k[l + 1];
            k[l] = std::min(a[l], cap(l));
        }
        a[0] = 2 * k[1];
    }
    int kmax = SL;
    for (int l = 1; l <= L; ++l) kmax = std::max(kmax, k[l]);
    const int r = std::min(KMAXC * SL, ((kmax + oversample + SL - 1) / SL) * SL);
    std::vector<int64_t> off(L + 2, 0), voff(L + 2, 0);
    for (int l = 1; l <= L; ++l) {
        off[l + 1] = off[l] + ((int64_t)1 << l) * a[l] * a[l];
        voff[l + 1] = voff[l] + ((int64_t)1 << l) * a[l];
    }
    const int64_t qtot = off[L + 1], vtot = voff[L + 1];
    // per-level buffer needs; gram chunking per level (children of level l)
    int64_t maxT = 1, maxQ = 1, maxSt = 1, maxB = 1, maxEig = 1, gpart = 1, amax = std::max(1, a[0]);
    std::vector<int> crows(L + 1, 256), cmx(L + 1, 1), rbl(L + 1, 1);
    for (int l = 1; l <= L; ++l) {
        const int64_t nodes = (int64_t)1 << l;
        maxT = std::max(maxT, nodes * a[l] * r);
        maxQ = std::max(maxQ, nodes * a[l] * a[l]);
        maxSt = std::max(maxSt, nodes * k[l] * r);
        maxB = std::max(maxB, (nodes / 2) * (int64_t)k[l] * k[l]);
        maxEig = std::max(maxEig, 2 * nodes * a[l]);
        amax = std::max(amax, (int64_t)a[l]);
        int64_t csz = 0;
        for (int64_t c = 0; c < nodes; ++c) csz = std::max(csz, bnd[boff(l) + c + 1] - bnd[boff(l) + c]);
        crows[l] = (int)std::max<int64_t>(256, cdiv(cdiv(csz, 64), 32) * 32);
        cmx[l] = (int)cdiv(csz, crows[l]);
        rbl[l] = (int)cdiv(csz, 64);
        gpart = std::max(gpart, (nodes / 2) * cmx[l] * (int64_t)(k[l] / SL) * (k[l] / SL) * SL * SL);
    }
    maxEig = std::max(maxEig, 2 * amax);
    maxQ = std::max(maxQ, amax * amax);  // the root block passes through Dn too
    int64_t maxV = std::max<int64_t>(amax, (int64_t)ell);  // the apply's temporary vector (nodes x a per level)
    for (int l = 1; l <= L; ++l) maxV = std::max(maxV, ((int64_t)1 << l) * a[l]);

    // device workspace (doubles, then int64, then int)
    const size_t nd = (size_t)n * m + 3 * (size_t)n * r + 3 * (size_t)n * kmax + 2 * (size_t)qtot +
                      (size_t)amax * amax + (size_t)maxT + 2 * (size_t)maxQ + 4 * (size_t)maxSt +
                      (size_t)(L + 1) * maxB + (size_t)gpart + 2 * (size_t)vtot + (size_t)leaves * ell +
                      2 * (size_t)amax + (size_t)maxV + (size_t)kHssPart + (size_t)maxEig + 256;
    const size_t nint = (size_t)n + bnd.size() + 16;
    const size_t nsmall = (size_t)std::max<int64_t>(leaves, 2) + 64;
    if (ensure(ctx, ctx->hss, sizeof(double) * nd + sizeof(int64_t) * nint + sizeof(int) * nsmall + 4096) != MAG_OK)
        return MAG_ENOMEM;
    double *p = (double *)ctx->hss.p;
    H.Xp = p; p += (size_t)n * m;
    double *Om = p; p += (size_t)n * r;
    double *S = p; p += (size_t)n * r;
    double *Tmp = p; p += (size_t)n * r;
    double *Ucur = p; p += (size_t)n * kmax;
    double *Unext = p; p += (size_t)n * kmax;
    double *Wz = p; p += (size_t)n * kmax;
    H.Q = p; p += qtot;
    H.Dt = p; p += qtot;
    H.Droot = p; p += (size_t)amax * amax;
    double *T = p; p += maxT;
    double *Dn = p; p += maxQ;
    double *T2 = p; p += maxQ;
    double *St[2] = {p, p + maxSt}; p += 2 * maxSt;
    double *Ot[2] = {p, p + maxSt}; p += 2 * maxSt;
    std::vector<double *> Bc(L + 1, nullptr);
    for (int l = 0; l <= L; ++l) { Bc[l] = p; p += maxB; }
    double *gp = p; p += gpart;
    H.ub = p; p += vtot;
    H.xb = p; p += vtot;
    H.xl = p; p += (size_t)leaves * ell;
    H.rr = p; p += 2 * (size_t)amax;
    H.tv = p; p += (size_t)maxV;
    H.part = p; p += (size_t)kHssPart;
    double *eigw = p; p += maxEig;
    p += 256;
    int64_t *ip = (int64_t *)p;
    H.perm = ip; ip += n;
    H.bnd = ip; ip += bnd.size();
    int *info = (int *)(ip + 8);
    H.n = n; H.npad = npad; H.m = m; H.L = L; H.ell = ell; H.t = t;
    H.k = k; H.a = a; H.off = off; H.voff = voff; H.blas = bh;

    if (hipMemcpyAsync(H.Xp, Xp.data(), sizeof(double) * n * m, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(H.perm, perm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(H.bnd, bnd.data(), sizeof(int64_t) * bnd.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MAG_EHIP;
    const int64_t *bL = H.bnd + boff(L);
    const double one = 1.0, mone = -1.0, zero = 0.0;
    auto check_info = [&](int count) -> int {
        std::vector<int> hi(count);
        if (hipMemcpyAsync(hi.data(), info, sizeof(int) * count, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MAG_EHIP;
        for (int v : hi)
            if (v != 0) return MAG_ENOTPD;
        return MAG_OK;
    };
    // Cholesky of each node's leading e x e block of D (ld a), retaken from the
    // copy in `src` with a growing diagonal shift when the compressed block is
    // not positive definite (it approximates a Schur complement of Z; the shift
    // only changes the preconditioner, GMRES keeps the exact products)
    H.shift = 0.0;
    auto potrf_shifted = [&](double *D, const double *src, int a, int e, int64_t nodes) -> int {
        for (int attempt = 0;; ++attempt) {
            RBCHK(rocsolver_dpotrf_strided_batched(bh, rocblas_fill_lower, e, D, a, (rocblas_stride)a * a, info,
                                                   (rocblas_int)nodes));
            const int rc = check_info((int)nodes);
            if (rc != MAG_ENOTPD) return rc;
            if (attempt >= 8) return MAG_ENOTPD;
            if (hipMemcpyAsync(D, src, sizeof(double) * nodes * a * a, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return MAG_EHIP;
            double *dmax = eigw;
            hipLaunchKernelGGL(k_hss_diagmax, dim3(1), dim3(NT), 0, s, D, a, e, nodes, dmax);
            double hmax = 0.0;
            if (hipMemcpyAsync(&hmax, dmax, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return MAG_EHIP;
            const double sigma = hmax * std::pow(10.0, -8.0 + attempt);
            hipLaunchKernelGGL(k_hss_shift, dim3(hss_grid(nodes * (int64_t)e)), dim3(NT), 0, s, D, a, e, nodes, sigma);
            H.shift = std::max(H.shift, sigma);
        }
    };

    if (L == 0) {
        // one leaf: the root block is Z itself
        hipLaunchKernelGGL(k_hss_leaf_block, dim3(hss_grid((int64_t)ell * ell)), dim3(NT), 0, s, H.Xp, m, t, bL, ell,
                           (int64_t)1, H.Droot);
        RBCHK(rocsolver_dpotrf(bh, rocblas_fill_lower, ell, H.Droot, ell, info));
        HSSCHK(check_info(1));  // exact Z: not positive definite only for coincident points
        // the apply multiplies by the factor's inverse
        RBCHK(rocsolver_dtrtri(bh, rocblas_fill_lower, rocblas_diagonal_non_unit, ell, H.Droot, ell, info));
        return check_info(1);
    }

    // 1. S = (Z - leaf blocks) Omega, from the sibling-pair products of every level
    hipLaunchKernelGGL(k_omega, dim3(2048), dim3(NT), 0, s, Om, n, r, r, mix64(seed + 0x2545f4914f6cdd1dull));
    launch_fill(s, S, (int64_t)n * r, 0.0);
    for (int l = 1; l <= L; ++l) {
        const int64_t tasks = (int64_t)1 << (l - 1);
        for (int mode = 0; mode < 2; ++mode)
            launch_zblock(s, H.Xp, m, t, H.bnd + boff(l), mode, tasks, rbl[l], Om, Tmp, r, r);
        launch_axpy1(s, Tmp, S, (int64_t)n * r);
    }
    // Bc[l][pair] = U(I_a)^T Z(I_a, I_b) U(I_b) for level l's sibling pairs, U: n x k[l]
    auto couplings = [&](const double *U, int l) {
        const int kl = k[l], nt = (kl / SL) * (kl / SL);
        const int64_t tasks = (int64_t)1 << (l - 1);
        launch_zblock(s, H.Xp, m, t, H.bnd + boff(l), 0, tasks, rbl[l], U, Wz, kl, kl);
        hipLaunchKernelGGL(k_gram_partial, dim3((unsigned)(tasks * cmx[l]), (unsigned)nt), dim3(NT), 0, s, U, kl, Wz,
                           kl, H.bnd + boff(l), 2, 0, crows[l], cmx[l], gp);
        hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)(tasks * nt), SL * SL / NT), dim3(NT), 0, s, gp, cmx[l], kl,
                           kl, Bc[l]);
    };

    // 2. leaves: bases from the eigenvectors of T T^T
    {
        const int kl = k[L];
        double *QL = H.Q + off[L];
        hipLaunchKernelGGL(k_hss_gather_rows, dim3(hss_grid(leaves * ell * (int64_t)r)), dim3(NT), 0, s, S, r, bL, ell,
                           leaves, T);
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_none, rocblas_operation_transpose, ell, ell, r, &one,
                                            T, ell, (rocblas_stride)ell * r, T, ell, (rocblas_stride)ell * r, &zero, QL,
                                            ell, (rocblas_stride)ell * ell, (rocblas_int)leaves));
        RBCHK(rocsolver_dsyevd_strided_batched(bh, rocblas_evect_original, rocblas_fill_lower, ell, QL, ell,
                                               (rocblas_stride)ell * ell, eigw, ell, eigw + leaves * ell, ell, info,
                                               (rocblas_int)leaves));
        HSSCHK(check_info((int)leaves));
        const double *V = QL + (int64_t)(ell - kl) * ell;
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_transpose, rocblas_operation_none, kl, r, ell, &one,
                                            V, ell, (rocblas_stride)ell * ell, T, ell, (rocblas_stride)ell * r, &zero,
                                            St[0], kl, (rocblas_stride)kl * r, (rocblas_int)leaves));
        hipLaunchKernelGGL(k_hss_gather_rows, dim3(hss_grid(leaves * ell * (int64_t)r)), dim3(NT), 0, s, Om, r, bL, ell,
                           leaves, T);
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_transpose, rocblas_operation_none, kl, r, ell, &one,
                                            V, ell, (rocblas_stride)ell * ell, T, ell, (rocblas_stride)ell * r, &zero,
                                            Ot[0], kl, (rocblas_stride)kl * r, (rocblas_int)leaves));
        hipLaunchKernelGGL(k_hss_scatter_basis, dim3(hss_grid(leaves * ell * (int64_t)kl)), dim3(NT), 0, s, QL, ell, kl,
                           bL, leaves, Ucur);
    }
    // 3. levels L-1 .. 1: couplings of the children, projected samples, nested bases
    int cur = 0;
    for (int l = L - 1; l >= 1; --l) {
        const int kc = k[l + 1], al = a[l], kl = k[l];
        const int64_t nodes = (int64_t)1 << l;
        couplings(Ucur, l + 1);
        // T = [S~_a - B O~_b ; S~_b - B^T O~_a]
        hipLaunchKernelGGL(k_hss_stack, dim3(hss_grid(nodes * al * (int64_t)r)), dim3(NT), 0, s, St[cur],
                           (int64_t)kc * r, kc, 0, kc, r, nodes, T);
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_none, rocblas_operation_none, kc, r, kc, &mone,
                                            Bc[l + 1], kc, (rocblas_stride)kc * kc, Ot[cur] + (int64_t)kc * r, kc,
                                            (rocblas_stride)2 * kc * r, &one, T, al, (rocblas_stride)al * r,
                                            (rocblas_int)nodes));
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_transpose, rocblas_operation_none, kc, r, kc, &mone,
                                            Bc[l + 1], kc, (rocblas_stride)kc * kc, Ot[cur], kc,
                                            (rocblas_stride)2 * kc * r, &one, T + kc, al, (rocblas_stride)al * r,
                                            (rocblas_int)nodes));
        double *Ql = H.Q + off[l];
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_none, rocblas_operation_transpose, al, al, r, &one,
                                            T, al, (rocblas_stride)al * r, T, al, (rocblas_stride)al * r, &zero, Ql, al,
                                            (rocblas_stride)al * al, (rocblas_int)nodes));
        RBCHK(rocsolver_dsyevd_strided_batched(bh, rocblas_evect_original, rocblas_fill_lower, al, Ql, al,
                                               (rocblas_stride)al * al, eigw, al, eigw + nodes * al, al, info,
                                               (rocblas_int)nodes));
        HSSCHK(check_info((int)nodes));
        const double *R = Ql + (int64_t)(al - kl) * al;
        const int nx = cur ^ 1;
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_transpose, rocblas_operation_none, kl, r, al, &one,
                                            R, al, (rocblas_stride)al * al, T, al, (rocblas_stride)al * r, &zero,
                                            St[nx], kl, (rocblas_stride)kl * r, (rocblas_int)nodes));
        hipLaunchKernelGGL(k_hss_stack, dim3(hss_grid(nodes * al * (int64_t)r)), dim3(NT), 0, s, Ot[cur],
                           (int64_t)kc * r, kc, 0, kc, r, nodes, T);
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_transpose, rocblas_operation_none, kl, r, al, &one,
                                            R, al, (rocblas_stride)al * al, T, al, (rocblas_stride)al * r, &zero,
                                            Ot[nx], kl, (rocblas_stride)kl * r, (rocblas_int)nodes));
        // explicit bases of level l: U_l(I_c) = U_{l+1}(I_c) R_c for each child c
        // (R_c copied out to kc x kl blocks in T2, then the row-block products)
        hipLaunchKernelGGL(k_hss_split_R, dim3(hss_grid(2 * nodes * (int64_t)kc * kl)), dim3(NT), 0, s, Ql, al, kl, kc,
                           nodes, T2);
        hipLaunchKernelGGL(k_rowmul, dim3((unsigned)(2 * nodes * rbl[l + 1]), (unsigned)(kl / SL)), dim3(NT), 0, s,
                           Ucur, kc, Unext, kl, T2, (int64_t)kc * kl, H.bnd + boff(l + 1), 1, 0, rbl[l + 1], 0);
        std::swap(Ucur, Unext);
        cur = nx;
    }
    couplings(Ucur, 1);

    // 4. ULV, bottom-up
    for (int l = L; l >= 1; --l) {
        const int al = a[l], kl = k[l], el = al - kl;
        const int64_t nodes = (int64_t)1 << l;
        double *Ql = H.Q + off[l], *Dl = H.Dt + off[l];
        if (l == L)
            hipLaunchKernelGGL(k_hss_leaf_block, dim3(hss_grid(nodes * (int64_t)al * al)), dim3(NT), 0, s, H.Xp, m, t,
                               bL, ell, nodes, Dn);
        else
            hipLaunchKernelGGL(k_hss_assemble, dim3(hss_grid(nodes * (int64_t)al * al)), dim3(NT), 0, s,
                               H.Dt + off[l + 1], a[l + 1], k[l + 1], Bc[l + 1], nodes, Dn);
        // Dt = Q^T D Q
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_none, rocblas_operation_none, al, al, al, &one, Dn,
                                            al, (rocblas_stride)al * al, Ql, al, (rocblas_stride)al * al, &zero, T2, al,
                                            (rocblas_stride)al * al, (rocblas_int)nodes));
        RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_transpose, rocblas_operation_none, al, al, al, &one,
                                            Ql, al, (rocblas_stride)al * al, T2, al, (rocblas_stride)al * al, &zero, Dl,
                                            al, (rocblas_stride)al * al, (rocblas_int)nodes));
        if (el > 0) {
            // keep Q^T D Q for a retake with a shift (Dn is free after the transform)
            if (hipMemcpyAsync(Dn, Dl, sizeof(double) * nodes * al * al, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return MAG_EHIP;
            HSSCHK(potrf_shifted(Dl, Dn, al, el, nodes));
            RBCHK(rocblas_dtrsm_strided_batched(bh, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                                                rocblas_diagonal_non_unit, kl, el, &one, Dl, al,
                                                (rocblas_stride)al * al, Dl + el, al, (rocblas_stride)al * al,
                                                (rocblas_int)nodes));
            RBCHK(rocblas_dgemm_strided_batched(bh, rocblas_operation_none, rocblas_operation_transpose, kl, kl, el,
                                                &mone, Dl + el, al, (rocblas_stride)al * al, Dl + el, al,
                                                (rocblas_stride)al * al, &one, Dl + el + (int64_t)el * al, al,
                                                (rocblas_stride)al * al, (rocblas_int)nodes));
        }
    }
    hipLaunchKernelGGL(k_hss_assemble, dim3(hss_grid((int64_t)a[0] * a[0])), dim3(NT), 0, s, H.Dt + off[1], a[1], k[1],
                       Bc[1], (int64_t)1, Dn);
    if (hipMemcpyAsync(H.Droot, Dn, sizeof(double) * a[0] * a[0], hipMemcpyDeviceToDevice, s) != hipSuccess)
        return MAG_EHIP;
    HSSCHK(potrf_shifted(H.Droot, Dn, a[0], a[0], 1));
    RBCHK(rocsolver_dtrtri(bh, rocblas_fill_lower, rocblas_diagonal_non_unit, a[0], H.Droot, a[0], info));
    HSSCHK(check_info(1));
    // 5. the eliminated blocks' factors L_e (and the root's) are only applied from
    // here on: keep their inverses in place, so the apply multiplies instead of
    // solving
    for (int l = L; l >= 1; --l) {
        const int al = a[l], el = al - k[l];
        if (el <= 0) continue;
        RBCHK(rocsolver_dtrtri_strided_batched(bh, rocblas_fill_lower, rocblas_diagonal_non_unit, el, H.Dt + off[l], al,
                                               (rocblas_stride)al * al, info, (rocblas_int)((int64_t)1 << l)));
        HSSCHK(check_info((int)((int64_t)1 << l)));
    }
    if (hipGetLastError() != hipSuccess) return MAG_EHIP;
    return MAG_OK;
}

int hss_apply(hipStream_t s, const HssFactor &H, const double *r, double *z)
{
    const int L = H.L, ell = H.ell;
    const int64_t leaves = (int64_t)1 << L;
    const int64_t *bL = H.bnd + boff(L);
    hipLaunchKernelGGL(k_hss_gather_vec, dim3(hss_grid(leaves * ell)), dim3(NT), 0, s, r, H.perm, bL, ell, leaves,
                       H.xl);
    if (L == 0) {
        // one leaf: x = R^{-T} R^{-1} r with the inverse R^{-1} of Z's Cholesky factor
        launch_bgemv_n(s, H.Droot, ell, 0, H.xl, 0, H.tv, 0, H.part, ell, ell, 1, 1.0, 0.0, true);
        launch_bgemv_t(s, H.Droot, ell, 0, H.tv, 0, H.xl, 0, ell, ell, 1, 1.0, 0.0, true);
        hipLaunchKernelGGL(k_hss_scatter_vec, dim3(hss_grid(std::max<int64_t>(leaves * ell, H.npad))), dim3(NT), 0, s,
                           H.xl, H.perm, bL, ell, leaves, H.n, H.npad, z);
        return hipGetLastError() == hipSuccess ? MAG_OK : MAG_EHIP;
    }
    // up: u = Q^T (node rhs); y_e = L_e^{-1} u_e (L_e^{-1} is stored); u_s -= W y_e
    for (int l = L; l >= 1; --l) {
        const int al = H.a[l], kl = H.k[l], el = al - kl;
        const int64_t nodes = (int64_t)1 << l;
        const double *rin;
        if (l == L) {
            rin = H.xl;
        } else {
            const int ac = H.a[l + 1];
            hipLaunchKernelGGL(k_hss_stack, dim3(hss_grid(nodes * al)), dim3(NT), 0, s, H.ub + H.voff[l + 1], (int64_t)ac,
                               ac, ac - H.k[l + 1], H.k[l + 1], 1, nodes, H.xb + H.voff[l]);
            rin = H.xb + H.voff[l];
        }
        double *u = H.ub + H.voff[l];
        const double *Ql = H.Q + H.off[l], *Dl = H.Dt + H.off[l];
        const int64_t sq = (int64_t)al * al;
        launch_bgemv_t(s, Ql, al, sq, rin, al, u, al, al, al, nodes, 1.0, 0.0, false);
        if (el > 0) {
            launch_bgemv_n(s, Dl, al, sq, u, al, H.tv, al, H.part, el, el, nodes, 1.0, 0.0, true);
            launch_bgemv_n(s, Dl + el, al, sq, H.tv, al, u + el, al, H.part, kl, el, nodes, -1.0, 1.0, false);
            hipLaunchKernelGGL(k_hss_copy_head, dim3(hss_grid(nodes * el)), dim3(NT), 0, s, H.tv, u, al, el, nodes);
        }
    }
    // root: x = R^{-T} R^{-1} b
    const int a0 = H.a[0];
    hipLaunchKernelGGL(k_hss_stack, dim3(hss_grid(a0)), dim3(NT), 0, s, H.ub + H.voff[1], (int64_t)H.a[1], H.a[1],
                       H.a[1] - H.k[1], H.k[1], 1, (int64_t)1, H.rr);
    launch_bgemv_n(s, H.Droot, a0, 0, H.rr, 0, H.tv, 0, H.part, a0, a0, 1, 1.0, 0.0, true);
    launch_bgemv_t(s, H.Droot, a0, 0, H.tv, 0, H.rr, 0, a0, a0, 1, 1.0, 0.0, true);
    // down: v = [y_e; x_s], x_e = L_e^{-T} (y_e - W^T x_s), x = Q v
    for (int l = 1; l <= L; ++l) {
        const int al = H.a[l], kl = H.k[l], el = al - kl;
        const int64_t nodes = (int64_t)1 << l;
        const double *xpar = (l == 1) ? H.rr : H.xb + H.voff[l - 1];
        const int apar = (l == 1) ? a0 : H.a[l - 1];
        double *v = H.ub + H.voff[l];  // y_e stays in place, x_s is written after it
        hipLaunchKernelGGL(k_hss_down_vec, dim3(hss_grid(nodes * al)), dim3(NT), 0, s, H.ub + H.voff[l], xpar, apar, al,
                           kl, nodes, v);
        const double *Ql = H.Q + H.off[l], *Dl = H.Dt + H.off[l];
        const int64_t sq = (int64_t)al * al;
        if (el > 0) {
            launch_bgemv_t(s, Dl + el, al, sq, v + el, al, v, al, kl, el, nodes, -1.0, 1.0, false);
            launch_bgemv_t(s, Dl, al, sq, v, al, H.tv, al, el, el, nodes, 1.0, 0.0, true);
            hipLaunchKernelGGL(k_hss_copy_head, dim3(hss_grid(nodes * el)), dim3(NT), 0, s, H.tv, v, al, el, nodes);
        }
        double *xo = (l == L) ? H.xl : H.xb + H.voff[l];
        launch_bgemv_n(s, Ql, al, sq, v, al, xo, al, H.part, al, al, nodes, 1.0, 0.0, false);
    }
    hipLaunchKernelGGL(k_hss_scatter_vec, dim3(hss_grid(std::max<int64_t>(leaves * ell, H.npad))), dim3(NT), 0, s, H.xl,
                       H.perm, bL, ell, leaves, H.n, H.npad, z);
    return hipGetLastError() == hipSuccess ? MAG_OK : MAG_EHIP;
}

}  // namespace mag
