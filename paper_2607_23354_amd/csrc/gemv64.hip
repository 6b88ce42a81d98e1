// gemv64.hip -- FP64 matrix-free product y = Z v with Z = exp[-t d]
// regenerated tile by tile from the coordinates (Section 2), used for the
// refinement residual r = 1 - Z w and for the Krylov matvecs.  Nothing of Z is
// stored: the cost is n^2 FP64 distance + exp evaluations, the traffic only
// O(n m).  The entry is formed exactly as the tile generator forms it
// (exact differences, uncontracted squared sum in ascending l, sqrt, then
// exp(-(t d))), in FP64.
//
// Single solves use the symmetry of Z: only the 128 x 128 tiles (I, J) with
// J <= I are evaluated; each off-diagonal tile adds Z_IJ v_J to block I and
// Z_IJ^T v_I to block J, so every entry is formed once.  Per-tile row and
// column sums go to a tile-major buffer and a second kernel adds them per
// block in a fixed order (deterministic), optionally forming b - Z v and its
// max-norm.  The batched path keeps the row-per-thread form: (row blocks of
// 256 rows) x (column splits), partial row sums split-major.
#include "internal.hpp"

#include <type_traits>

#include <algorithm>
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
                    const double z = (k0 + c == j) ? 1.0 : zexp(t, s);
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
                    const double z = (k0 + c == j) ? 1.0 : zexp(t, s);
                    acc = fma(z, vc[c], acc);
                }
            }
        }
    }
    if (j < npad) partial[by * npad + j] = live ? acc : 0.0;
}

// Table-driven exp for the symmetric products (Tang, "Table-driven
// implementation of the exponential function in IEEE floating-point
// arithmetic", ACM TOMS 15, 1989): x = (64 e + j) ln2/64 + r with |r| <= ln2/128,
// e^x = 2^e 2^(j/64) e^r, 2^(j/64) from a double-double table and e^r - 1 from
// its Taylor series to degree 5 (truncation below 4e-17 on that interval);
// about 12 FP64 operations against the 20 of exp_nonpos.  The table
// (gen_exp2_table.py): 2^(j/64) rounded to double, then the rounded remainder.
__device__ const double kExp2Tab[128] = {
    0x1.0000000000000p+0, 0x0.0p+0,
    0x1.02c9a3e778061p+0, -0x1.19083535b085dp-56,
    0x1.059b0d3158574p+0, 0x1.d73e2a475b465p-55,
    0x1.0874518759bc8p+0, 0x1.186be4bb284ffp-57,
    0x1.0b5586cf9890fp+0, 0x1.8a62e4adc610bp-54,
    0x1.0e3ec32d3d1a2p+0, 0x1.03a1727c57b53p-59,
    0x1.11301d0125b51p+0, -0x1.6c51039449b3ap-54,
    0x1.1429aaea92de0p+0, -0x1.32fbf9af1369ep-54,
    0x1.172b83c7d517bp+0, -0x1.19041b9d78a76p-55,
    0x1.1a35beb6fcb75p+0, 0x1.e5b4c7b4968e4p-55,
    0x1.1d4873168b9aap+0, 0x1.e016e00a2643cp-54,
    0x1.2063b88628cd6p+0, 0x1.dc775814a8495p-55,
    0x1.2387a6e756238p+0, 0x1.9b07eb6c70573p-54,
    0x1.26b4565e27cddp+0, 0x1.2bd339940e9d9p-55,
    0x1.29e9df51fdee1p+0, 0x1.612e8afad1255p-55,
    0x1.2d285a6e4030bp+0, 0x1.0024754db41d5p-54,
    0x1.306fe0a31b715p+0, 0x1.6f46ad23182e4p-55,
    0x1.33c08b26416ffp+0, 0x1.32721843659a6p-54,
    0x1.371a7373aa9cbp+0, -0x1.63aeabf42eae2p-54,
    0x1.3a7db34e59ff7p+0, -0x1.5e436d661f5e3p-56,
    0x1.3dea64c123422p+0, 0x1.ada0911f09ebcp-55,
    0x1.4160a21f72e2ap+0, -0x1.ef3691c309278p-58,
    0x1.44e086061892dp+0, 0x1.89b7a04ef80d0p-59,
    0x1.486a2b5c13cd0p+0, 0x1.3c1a3b69062f0p-56,
    0x1.4bfdad5362a27p+0, 0x1.d4397afec42e2p-56,
    0x1.4f9b2769d2ca7p+0, -0x1.4b309d25957e3p-54,
    0x1.5342b569d4f82p+0, -0x1.07abe1db13cadp-55,
    0x1.56f4736b527dap+0, 0x1.9bb2c011d93adp-54,
    0x1.5ab07dd485429p+0, 0x1.6324c054647adp-54,
    0x1.5e76f15ad2148p+0, 0x1.ba6f93080e65ep-54,
    0x1.6247eb03a5585p+0, -0x1.383c17e40b497p-54,
    0x1.6623882552225p+0, -0x1.bb60987591c34p-54,
    0x1.6a09e667f3bcdp+0, -0x1.bdd3413b26456p-54,
    0x1.6dfb23c651a2fp+0, -0x1.bbe3a683c88abp-57,
    0x1.71f75e8ec5f74p+0, -0x1.16e4786887a99p-55,
    0x1.75feb564267c9p+0, -0x1.0245957316dd3p-54,
    0x1.7a11473eb0187p+0, -0x1.41577ee04992fp-55,
    0x1.7e2f336cf4e62p+0, 0x1.05d02ba15797ep-56,
    0x1.82589994cce13p+0, -0x1.d4c1dd41532d8p-54,
    0x1.868d99b4492edp+0, -0x1.fc6f89bd4f6bap-54,
    0x1.8ace5422aa0dbp+0, 0x1.6e9f156864b27p-54,
    0x1.8f1ae99157736p+0, 0x1.5cc13a2e3976cp-55,
    0x1.93737b0cdc5e5p+0, -0x1.75fc781b57ebcp-57,
    0x1.97d829fde4e50p+0, -0x1.d185b7c1b85d1p-54,
    0x1.9c49182a3f090p+0, 0x1.c7c46b071f2bep-56,
    0x1.a0c667b5de565p+0, -0x1.359495d1cd533p-54,
    0x1.a5503b23e255dp+0, -0x1.d2f6edb8d41e1p-54,
    0x1.a9e6b5579fdbfp+0, 0x1.0fac90ef7fd31p-54,
    0x1.ae89f995ad3adp+0, 0x1.7a1cd345dcc81p-54,
    0x1.b33a2b84f15fbp+0, -0x1.2805e3084d708p-57,
    0x1.b7f76f2fb5e47p+0, -0x1.5584f7e54ac3bp-56,
    0x1.bcc1e904bc1d2p+0, 0x1.23dd07a2d9e84p-55,
    0x1.c199bdd85529cp+0, 0x1.11065895048ddp-55,
    0x1.c67f12e57d14bp+0, 0x1.2884dff483cadp-54,
    0x1.cb720dcef9069p+0, 0x1.503cbd1e949dbp-56,
    0x1.d072d4a07897cp+0, -0x1.cbc3743797a9cp-54,
    0x1.d5818dcfba487p+0, 0x1.2ed02d75b3707p-55,
    0x1.da9e603db3285p+0, 0x1.c2300696db532p-54,
    0x1.dfc97337b9b5fp+0, -0x1.1a5cd4f184b5cp-54,
    0x1.e502ee78b3ff6p+0, 0x1.39e8980a9cc8fp-55,
    0x1.ea4afa2a490dap+0, -0x1.e9c23179c2893p-54,
    0x1.efa1bee615a27p+0, 0x1.dc7f486a4b6b0p-54,
    0x1.f50765b6e4540p+0, 0x1.9d3e12dd8a18bp-54,
    0x1.fa7c1819e90d8p+0, 0x1.74853f3a5931ep-55,
};

// exp(x) for x <= 0 with the table T (64 (hi, lo) pairs, in LDS); the result
// underflows to 0 below about -745
__device__ __forceinline__ double exp_tab(double x, const double2 *T)
{
    x = fmax(x, -1.0e4);
    const double kd = rint(x * 0x1.71547652b82fep+6);  // 64 / ln2
    double r = fma(-kd, 0x1.62e42fee00000p-7, x);      // ln2/64, 33-bit head: k head is exact
    r = fma(-kd, 0x1.a39ef35793c76p-39, r);            // and its tail
    const int k = (int)kd;
    double q = fma_uc(1.0 / 120.0, r, 1.0 / 24.0);
    q = fma_uc(q, r, 1.0 / 6.0);
    q = fma(q, r, 0.5);
    q = fma(q, r, 1.0);
    const double p = q * r;  // e^r - 1
    const double2 tj = T[k & 63];
    return ldexp(tj.x + fma(tj.x, p, tj.y), k >> 6);
}

__device__ __forceinline__ double zexp_tab(double t, double s, const double2 *T)
{
    return exp_tab(-(t * sqrt_pos(fmin(fmax(s, 1.0e-300), 1.0e300))), T);
}

constexpr int TS = 128;       // symmetric tile edge
constexpr int kEntExp = 0, kEntExp32 = 1, kEntShiftDist = 2;
constexpr int MMAX_SYM = 16;  // largest dimension of the symmetric product

// Lower tile index -> (I, J), J <= I, idx = I (I + 1) / 2 + J.
__device__ inline void tri_tile(int64_t idx, int64_t &I, int64_t &J)
{
    int64_t r = (int64_t)((sqrt(8.0 * (double)idx + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > idx) --r;
    while ((r + 1) * (r + 2) / 2 <= idx) ++r;
    I = r;
    J = idx - r * (r + 1) / 2;
}

// One lower tile (I, J) of Z per workgroup; thread (ty, tx) owns rows 8 ty ..
// and columns 8 tx .. of the tile.  part[tile * 2 TS + p]: row sums
// sum_c Z(r0 + p, c) v_c over the tile's columns; part[tile * 2 TS + TS + p]:
// column sums sum_r Z(r, c0 + p) v_r (off-diagonal tiles only; a diagonal
// tile is summed over its full square as rows).  M > 0: compile-time m.
// ENT: the entry, kEntExp exp(-t d) in FP64, kEntExp32 the same in FP32 (sums in
// FP64), kEntShiftDist t - d in FP64 (t carries the shift c of the scale-zero
// system, diagonal c).
template <int M, int ENT = kEntExp>
__device__ __forceinline__ void zmv_sym_body(const double *__restrict__ X, int64_t n, int m_rt, double t,
                                             const double *__restrict__ v, double *__restrict__ part,
                                             int64_t tile)
{
    constexpr int MM = (M > 0) ? M : MMAX_SYM;
    __shared__ double Xr[MM][TS];
    __shared__ double Xc[MM][TS];
    __shared__ double vr[TS], vc[TS];
    __shared__ double red[4][TS];
    __shared__ double2 etab[64];
    const int m = (M > 0) ? M : m_rt;
    int64_t I, J;
    tri_tile(tile, I, J);
    const int64_t r0 = I * TS, c0 = J * TS;
    const bool diag = (I == J);
    const int tid = threadIdx.x;
    for (int e = tid; e < m * TS; e += 256) {
        const int l = e / TS, p = e % TS;
        Xr[l][p] = (r0 + p < n) ? X[(r0 + p) * m + l] : 0.0;
        Xc[l][p] = (c0 + p < n) ? X[(c0 + p) * m + l] : 0.0;
    }
    if (tid < TS) {
        vr[tid] = (r0 + tid < n) ? v[r0 + tid] : 0.0;
        vc[tid] = (c0 + tid < n) ? v[c0 + tid] : 0.0;
    }
    if (tid < 64) etab[tid] = make_double2(kExp2Tab[2 * tid], kExp2Tab[2 * tid + 1]);
    __syncthreads();
    const int ty = tid >> 4, tx = tid & 15;
    const int nr = (int)min((int64_t)TS, n - r0), nc = (int)min((int64_t)TS, n - c0);
    double xr[8][(M > 0) ? M : 1];
    if (M > 0) {
#pragma unroll
        for (int ii = 0; ii < 8; ++ii)
#pragma unroll
            for (int l = 0; l < ((M > 0) ? M : 1); ++l) xr[ii][l] = Xr[l][8 * ty + ii];
    }
    double rowacc[8], colsum[8];
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) rowacc[ii] = 0.0;
    // one column at a time: the 8 row entries of a column are independent
    // exp evaluations, enough parallelism without unrolling the columns.
    // Every entry is evaluated (padding coordinates are zero, the diagonal's
    // s = 0 is harmless) and, in diagonal and edge tiles only, then selected,
    // so the row entries stay independent straight-line code.
    auto columns = [&](auto full_tile) {
        constexpr bool FULL = decltype(full_tile)::value;
#pragma unroll 1
        for (int jj = 0; jj < 8; ++jj) {
            const int c = 8 * tx + jj;
            double xc[MM];
#pragma unroll
            for (int l = 0; l < MM; ++l) xc[l] = (l < m) ? Xc[l][c] : 0.0;
            const double vcj = vc[c];
            double colacc = 0.0;
#pragma unroll
            for (int ii = 0; ii < 8; ++ii) {
                const int r = 8 * ty + ii;
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < MM; ++l) {
                    if (l < m) {
                        const double xrv = (M > 0) ? xr[ii][(M > 0) ? l : 0] : Xr[l][r];
                        s = sq_acc(s, xrv - xc[l]);
                    }
                }
                double z;
                if (ENT == kEntExp32) z = (double)expf(-((float)t * sqrtf((float)s)));  // entry in FP32, sums in FP64
                else if (ENT == kEntShiftDist) z = t - sqrt(s);
                else z = zexp_tab(t, s, etab);
                if (!FULL) {
                    z = (diag && r == c) ? ((ENT == kEntShiftDist) ? t : 1.0) : z;
                    z = (r < nr && c < nc) ? z : 0.0;
                }
                rowacc[ii] = fma(z, vcj, rowacc[ii]);
                colacc = fma(z, vr[r], colacc);
            }
            colsum[jj] = colacc;
        }
    };
    if (!diag && nr == TS && nc == TS)  // uniform per workgroup
        columns(std::true_type{});
    else
        columns(std::false_type{});
    double *pt = part + tile * 2 * TS;
    // rows: sum over the 16 tx lanes (contiguous) by a fixed butterfly
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) {
        double a = rowacc[ii];
        a += __shfl_xor(a, 1);
        a += __shfl_xor(a, 2);
        a += __shfl_xor(a, 4);
        a += __shfl_xor(a, 8);
        rowacc[ii] = a;
    }
    if (tx == 0) {
#pragma unroll
        for (int ii = 0; ii < 8; ++ii) pt[8 * ty + ii] = rowacc[ii];
    }
    if (diag) return;  // uniform per workgroup
    // columns: sum over the 4 ty of a wave (lanes 16 and 32 apart), then the 4 waves
    const int wave = tid >> 6, tyw = (tid >> 4) & 3;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
        double a = colsum[jj];
        a += __shfl_xor(a, 16);
        a += __shfl_xor(a, 32);
        colsum[jj] = a;
    }
    if (tyw == 0) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) red[wave][8 * tx + jj] = colsum[jj];
    }
    __syncthreads();
    if (tid < TS) pt[TS + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// Block I of y (rows r0 .. r0 + TS): sum of the row sums of tiles (I, 0..I)
// and the column sums of tiles (I+1..T-1, I), in that order.  mode 0: y = Z v;
// mode 1: y = b - Z v (b == NULL: ones) and blkmax[I] = max |y| over the block.
// m <= 3: the entry loop fits 128 VGPRs, so four workgroups share a CU (more
// waves to hide the FP64 latency); larger m keeps its coordinates in registers.
template <int M, int ENT = kEntExp>
__global__ void __launch_bounds__(256, (M >= 1 && M <= 3) ? 4 : 1)
k_zmv_sym(const double *__restrict__ X, int64_t n, int m_rt, double t, const double *__restrict__ v,
          double *__restrict__ part)
{
    zmv_sym_body<M, ENT>(X, n, m_rt, t, v, part, blockIdx.x);
}

__device__ __forceinline__ void zmv_sym_reduce_body(const double *__restrict__ part, int64_t T, int64_t n,
                                                    int64_t npad, double *__restrict__ y,
                                                    const double *__restrict__ b, int mode,
                                                    double *__restrict__ blkmax, int64_t I)
{
    __shared__ double red[TS];
    const int p = threadIdx.x;
    const int64_t row = I * TS + p;
    double s = 0.0;
    const int64_t base = I * (I + 1) / 2;
    for (int64_t Jt = 0; Jt <= I; ++Jt) s += part[(base + Jt) * 2 * TS + p];
    for (int64_t It = I + 1; It < T; ++It) s += part[(It * (It + 1) / 2 + I) * 2 * TS + TS + p];
    double val = 0.0;
    if (row < n) val = (mode == 0) ? s : (b ? b[row] : 1.0) - s;
    if (row < npad) y[row] = val;
    if (mode == 1) {
        red[p] = fabs(val);
        __syncthreads();
        for (int w = TS / 2; w > 0; w >>= 1) {
            if (p < w) red[p] = fmax(red[p], red[p + w]);
            __syncthreads();
        }
        if (p == 0) blkmax[I] = red[0];
    }
}

__global__ void __launch_bounds__(TS)
k_zmv_sym_reduce(const double *__restrict__ part, int64_t T, int64_t n, int64_t npad, double *__restrict__ y,
                 const double *__restrict__ b, int mode, double *__restrict__ blkmax)
{
    zmv_sym_reduce_body(part, T, n, npad, y, b, mode, blkmax, blockIdx.x);
}

// Batched symmetric Z v: units T(T+1)/2 tiles per problem (T = npad / TS),
// then the per-block reduce (units T per problem); blkmax after the tiles.
template <int M>
__global__ void __launch_bounds__(256, (M >= 1 && M <= 3) ? 4 : 1) k_zmv_sym_b(const BProb *__restrict__ P, BWork w, int v_slot)
{
    const int i = bfind(w.pref, w.na, blockIdx.x);
    const BProb &q = P[w.plist[i]];
    if (!q.active) return;
    zmv_sym_body<M>(q.X, q.n, q.m, q.t, q.vec + (int64_t)v_slot * q.npad, q.partial, blockIdx.x - w.pref[i]);
}

__global__ void __launch_bounds__(TS)
k_zmv_sym_reduce_b(const BProb *__restrict__ P, BWork w, int y_slot, int b_slot, int mode)
{
    const int i = bfind(w.pref, w.na, blockIdx.x);
    const BProb &q = P[w.plist[i]];
    if (!q.active) return;
    const int64_t T = q.npad / TS;
    zmv_sym_reduce_body(q.partial, T, q.n, q.npad, q.vec + (int64_t)y_slot * q.npad,
                        b_slot >= 0 ? q.vec + (int64_t)b_slot * q.npad : nullptr, mode,
                        q.partial + T * (T + 1) / 2 * 2 * TS, blockIdx.x - w.pref[i]);
}

__global__ void __launch_bounds__(256) k_max_final_sym_b(const BProb *__restrict__ P, BWork w, int64_t out_off)
{
    __shared__ double red[256];
    const BProb &q = P[w.plist[blockIdx.x]];
    if (!q.active) return;
    const int64_t T = q.npad / TS;
    const double *blkmax = q.partial + T * (T + 1) / 2 * 2 * TS;
    double v = 0.0;
    for (int64_t e = threadIdx.x; e < T; e += 256) v = fmax(v, blkmax[e]);
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s2]);
        __syncthreads();
    }
    if (threadIdx.x == 0) q.scal[out_off] = red[0];
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
    if (!q.active) return;
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
    const int64_t T = (p.npad + TS - 1) / TS;
    const size_t sym = (size_t)(T * (T + 1) / 2) * 2 * TS + (size_t)T + 8;
    return std::max(sym, (size_t)(p.splits * p.npad + p.npad / 256 + 8));
}

int64_t zmv_b_units(int64_t n, int m)
{
    if (m <= MMAX_SYM) {
        const int64_t T = ((n + kPad - 1) / kPad * kPad) / TS;
        return T * (T + 1) / 2;
    }
    Plan p = plan_for(n);
    return p.rowblocks * p.splits;
}

int64_t zmv_b_reduce_units(int64_t n, int m)
{
    const int64_t npad = (n + kPad - 1) / kPad * kPad;
    return m <= MMAX_SYM ? npad / TS : npad / 256;
}

// Batched y_slot = Z v_slot (mode 0) or y_slot = b - Z v_slot with its max norm
// into scal[norm_off] (mode 1).  wz: units zmv_b_units(n, m); wr: units
// zmv_b_reduce_units(n, m).
void launch_zmv_b(hipStream_t s, int m, const BProb *P, const BWork &wz, const BWork &wr,
                  int v_slot, int y_slot, int b_slot, int mode, int64_t norm_off)
{
    if (wz.na <= 0) return;
    const dim3 g((unsigned)wz.total);
    if (m <= MMAX_SYM) {
        switch (m) {
        case 1: hipLaunchKernelGGL(k_zmv_sym_b<1>, g, dim3(256), 0, s, P, wz, v_slot); break;
        case 2: hipLaunchKernelGGL(k_zmv_sym_b<2>, g, dim3(256), 0, s, P, wz, v_slot); break;
        case 3: hipLaunchKernelGGL(k_zmv_sym_b<3>, g, dim3(256), 0, s, P, wz, v_slot); break;
        case 4: hipLaunchKernelGGL(k_zmv_sym_b<4>, g, dim3(256), 0, s, P, wz, v_slot); break;
        case 8: hipLaunchKernelGGL(k_zmv_sym_b<8>, g, dim3(256), 0, s, P, wz, v_slot); break;
        default: hipLaunchKernelGGL(k_zmv_sym_b<0>, g, dim3(256), 0, s, P, wz, v_slot); break;
        }
        hipLaunchKernelGGL(k_zmv_sym_reduce_b, dim3((unsigned)wr.total), dim3(TS), 0, s, P, wr, y_slot, b_slot, mode);
        if (mode == 1)
            hipLaunchKernelGGL(k_max_final_sym_b, dim3(wz.na), dim3(256), 0, s, P, wz, norm_off);
        return;
    }
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

size_t zmv_split_partial_doubles(int64_t n)
{
    Plan p = plan_for(n);
    return (size_t)(p.splits * p.npad + p.npad / 256);
}

// Row-per-thread form (any m): (row blocks) x (column splits), then the split reduce.
void launch_zmv_split(hipStream_t s, const double *X, int64_t n, int m, double t, const double *v,
                             double *y, const double *b, int mode, double *partial, double *out_norm)
{
    Plan p = plan_for(n);
    dim3 grid((unsigned)p.rowblocks, (unsigned)p.splits);
    hipLaunchKernelGGL(k_zmv_partial<0>, grid, dim3(RT), 0, s, X, n, m, t, v, partial, p.cps, p.npad);
    const int64_t rb = p.npad / 256;
    double *blkmax = partial + p.splits * p.npad;
    hipLaunchKernelGGL(k_zmv_reduce, dim3((unsigned)rb), dim3(256), 0, s, partial, p.npad, n, (int)p.splits, y, b,
                       mode, blkmax);
    if (mode == 1 && out_norm)
        hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, blkmax, rb, out_norm);
}

template <int ENT>
void launch_zmv_sym_tiles(hipStream_t s, const double *X, int64_t n, int m, double t, const double *v,
                          double *partial, const dim3 grid)
{
    switch (m) {
    case 1: hipLaunchKernelGGL((k_zmv_sym<1, ENT>), grid, dim3(256), 0, s, X, n, m, t, v, partial); break;
    case 2: hipLaunchKernelGGL((k_zmv_sym<2, ENT>), grid, dim3(256), 0, s, X, n, m, t, v, partial); break;
    case 3: hipLaunchKernelGGL((k_zmv_sym<3, ENT>), grid, dim3(256), 0, s, X, n, m, t, v, partial); break;
    case 4: hipLaunchKernelGGL((k_zmv_sym<4, ENT>), grid, dim3(256), 0, s, X, n, m, t, v, partial); break;
    case 8: hipLaunchKernelGGL((k_zmv_sym<8, ENT>), grid, dim3(256), 0, s, X, n, m, t, v, partial); break;
    default: hipLaunchKernelGGL((k_zmv_sym<0, ENT>), grid, dim3(256), 0, s, X, n, m, t, v, partial); break;
    }
}

void launch_zmv(hipStream_t s, const double *X, int64_t n, int m, double t, const double *v,
                double *y, const double *b, int mode, double *partial, double *out_norm, bool f32_entries,
                int kernel)
{
    if (kernel == kKernShiftDist) {
        // the scale-zero system (m <= 16 only, checked by the caller)
        const int64_t npad = (n + kPad - 1) / kPad * kPad;
        const int64_t T = npad / TS;
        const int64_t tiles = T * (T + 1) / 2;
        launch_zmv_sym_tiles<kEntShiftDist>(s, X, n, m, t, v, partial, dim3((unsigned)tiles));
        double *blkmax = partial + tiles * 2 * TS;
        hipLaunchKernelGGL(k_zmv_sym_reduce, dim3((unsigned)T), dim3(TS), 0, s, partial, T, n, npad, y, b, mode,
                           blkmax);
        if (mode == 1 && out_norm)
            hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, blkmax, T, out_norm);
        return;
    }
    if (m > MMAX_SYM) {
        launch_zmv_split(s, X, n, m, t, v, y, b, mode, partial, out_norm);
        return;
    }
    const int64_t npad = (n + kPad - 1) / kPad * kPad;
    const int64_t T = npad / TS;
    const int64_t tiles = T * (T + 1) / 2;
    const dim3 grid((unsigned)tiles);
    if (f32_entries) launch_zmv_sym_tiles<kEntExp32>(s, X, n, m, t, v, partial, grid);
    else launch_zmv_sym_tiles<kEntExp>(s, X, n, m, t, v, partial, grid);
    double *blkmax = partial + tiles * 2 * TS;
    hipLaunchKernelGGL(k_zmv_sym_reduce, dim3((unsigned)T), dim3(TS), 0, s, partial, T, n, npad, y, b, mode,
                       blkmax);
    if (mode == 1 && out_norm)
        hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, blkmax, T, out_norm);
}

}  // namespace mag
