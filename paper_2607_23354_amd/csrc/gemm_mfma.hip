// gemm_mfma.hip -- FP32 MFMA kernel for the Cholesky's dense contractions.
//
//   C (M x N)  <-  C - P Q^T      (kGemmSub: trailing SYRK/GEMM updates)
//   C (M x N)  <-  P Q^T          (kGemmSet: panel TRSM against an explicit
//                                   inverse of the diagonal block)
//   kGemmSetT: as kGemmSet and also C^T into CT (CT(j, i) = CT[i * ldc + j]),
//   staged through LDS so both stores are coalesced; the factorisation uses
//   it to keep L^T in the upper triangle for the backward substitution.
//
// All operands are column-major FP32: P(i, p) = P[p * ldp + i],
// Q(j, p) = Q[p * ldq + j], C(i, j) = C[j * ldc + i].  Accumulation is FP32
// on v_mfma_f32_32x32x2_f32.
//
// Workgroup tile 128 x 128, 4 waves in a 2 x 2 arrangement, each wave a
// 64 x 64 sub-tile held as 2 x 2 MFMA 32 x 32 accumulators (64 registers).
// The MFMA's A operand is taken from Q and its B operand from P, so an
// accumulator lane maps to a row i of C: each accumulator register is a
// 128-byte contiguous column segment for a half-wave, which makes both the
// initial load of C and the final store coalesced.
// K is staged through LDS in chunks of 16 by direct global-to-LDS loads,
// double-buffered, one barrier per stage; the accumulators start at zero and
// C is updated in the epilogue.
#include "internal.hpp"

namespace mag {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(1))) void *gptr;  // global operand of a direct LDS load
typedef __attribute__((address_space(3))) void *lptr;        // its LDS destination

constexpr int BT = 128;
constexpr int KC = 16;
constexpr int NT = 256;
constexpr int kXcds = 8;

__device__ inline void tri_index(int64_t idx, int64_t &ti, int64_t &tj)
{
    int64_t r = (int64_t)((sqrt(8.0 * (double)idx + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > idx) --r;
    while ((r + 1) * (r + 2) / 2 <= idx) ++r;
    ti = r;
    tj = idx - r * (r + 1) / 2;
}

constexpr int TLD = BT + 1;
// operand stages (2 buffers x P, Q); the SetT epilogue's transposed half tile needs a
// little more.  32 KB for the other modes lets four workgroups share a CU's LDS.
constexpr int LDS_STAGES = 2 * 2 * KC * BT;
constexpr int LDS_SETT = (LDS_STAGES > BT * (64 + 1)) ? LDS_STAGES : BT * (64 + 1);

template <int MODE, bool LDS_EPI = false>
__device__ __forceinline__ void gemm_tile_body(float *__restrict__ C, int64_t ldc,
                                               const float *__restrict__ P, int64_t ldp,
                                               const float *__restrict__ Q, int64_t ldq,
                                               int64_t ti, int64_t tj, int64_t K,
                                               float *__restrict__ CT)
{
    __shared__ float lds[MODE == kGemmSetT ? LDS_SETT : LDS_STAGES];
    float (*Ps)[KC][BT] = reinterpret_cast<float (*)[KC][BT]>(lds);
    float (*Qs)[KC][BT] = reinterpret_cast<float (*)[KC][BT]>(lds + 2 * KC * BT);
    const int64_t i0 = ti * BT, j0 = tj * BT;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wi = (wave & 1) * 64;
    const int wj = (wave >> 1) * 64;
    const int l32 = lane & 31;
    const int hi = lane >> 5;

    // accumulate P Q^T from zero; C is read only in the epilogue, which keeps the
    // stage loop free of waits on loads other than the operand prefetch
    v16f acc[2][2];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[jb][ib][r] = 0.0f;

    // global -> LDS staging by direct loads (global_load_lds_dwordx4): thread t
    // fetches the float4 at row 4 (t % 32), k = t / 32 (and k + 8), and a wave's
    // 64 lanes land as one contiguous 1 KB block, rows 2 w and 2 w + 1 of a stage
    const int lr = 4 * (threadIdx.x & 31);
    const int lp = threadIdx.x >> 5;
    const float *pg0 = P + lp * ldp + i0 + lr, *pg1 = P + (lp + 8) * ldp + i0 + lr;
    const float *qg0 = Q + lp * ldq + j0 + lr, *qg1 = Q + (lp + 8) * ldq + j0 + lr;
    const int64_t stepP = KC * ldp, stepQ = KC * ldq;
    const int w2 = 2 * __builtin_amdgcn_readfirstlane(wave);
    auto stage_in = [&](int b) {
        __builtin_amdgcn_global_load_lds((gptr)pg0, (lptr)&Ps[b][w2][0], 16, 0, 0);
        __builtin_amdgcn_global_load_lds((gptr)pg1, (lptr)&Ps[b][w2 + 8][0], 16, 0, 0);
        __builtin_amdgcn_global_load_lds((gptr)qg0, (lptr)&Qs[b][w2][0], 16, 0, 0);
        __builtin_amdgcn_global_load_lds((gptr)qg1, (lptr)&Qs[b][w2 + 8][0], 16, 0, 0);
    };
    stage_in(0);
    __syncthreads();

    const int nst = (int)(K / KC);
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        if (st + 1 < nst) {
            // the other buffer was last read before the previous barrier
            pg0 += stepP;
            pg1 += stepP;
            qg0 += stepQ;
            qg1 += stepQ;
            stage_in(buf ^ 1);
        }
#pragma unroll
        for (int kp = 0; kp < KC / 2; ++kp) {
            const int p = 2 * kp + hi;
            const float q0 = Qs[buf][p][wj + l32];
            const float q1 = Qs[buf][p][wj + 32 + l32];
            const float p0 = Ps[buf][p][wi + l32];
            const float p1 = Ps[buf][p][wi + 32 + l32];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(q0, p0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(q0, p1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(q1, p0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(q1, p1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();  // waits for the direct loads of the next stage too
    }

    if (MODE == kGemmSub && LDS_EPI) {
        // C -= acc through LDS (free after the last stage's barrier): 16 columns of the
        // wave's 64 x 64 quadrant at a time, written in the accumulator layout and read
        // back as 4 consecutive rows per lane, so C moves in float4 accesses.  Column
        // stride 72 keeps both halves of the wave on distinct banks.  (Short-K updates,
        // bound by their latency, take the direct epilogue below.)
        float *Tw = lds + wave * (16 * 72);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int jb = q >> 1, rq = q & 1;
#pragma unroll
            for (int rr = 0; rr < 8; ++rr) {
                const int r = 8 * rq + rr;
                const int c16 = 8 * (rr >> 2) + 4 * hi + (r & 3);
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) Tw[c16 * 72 + 32 * ib + l32] = acc[jb][ib][r];
            }
#pragma unroll
            for (int rd = 0; rd < 4; ++rd) {
                const int c16 = 4 * rd + (lane >> 4);
                const float4 a = *reinterpret_cast<const float4 *>(&Tw[c16 * 72 + 4 * (lane & 15)]);
                float4 *cp = reinterpret_cast<float4 *>(C + (j0 + wj + 32 * jb + 16 * rq + c16) * ldc + i0 + wi +
                                                        4 * (lane & 15));
                float4 c = *cp;
                c.x -= a.x;
                c.y -= a.y;
                c.z -= a.z;
                c.w -= a.w;
                *cp = c;
            }
        }
    } else {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int ib = 0; ib < 2; ++ib) {
                const int64_t i = i0 + wi + ib * 32 + l32;
                if (MODE == kGemmSub) {
                    float cv[16];
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int64_t j = j0 + wj + jb * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
                        cv[r] = C[j * ldc + i];
                    }
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int64_t j = j0 + wj + jb * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
                        C[j * ldc + i] = cv[r] - acc[jb][ib][r];
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int64_t j = j0 + wj + jb * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
                        C[j * ldc + i] = acc[jb][ib][r];
                    }
                }
            }
    }
    if (MODE == kGemmSetT) {
        // transposed copy, 64 columns of the tile at a time through LDS (T[jl][i])
        float *T = lds;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            __syncthreads();
            if ((wave >> 1) == half) {
#pragma unroll
                for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib) {
                        const int il = wi + ib * 32 + l32;
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int jl = jb * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
                            T[jl * (BT + 1) + il] = acc[jb][ib][r];
                        }
                    }
            }
            __syncthreads();
            const int jl = threadIdx.x & 63;
            for (int il = threadIdx.x >> 6; il < BT; il += NT / 64)
                CT[(i0 + il) * ldc + j0 + half * 64 + jl] = T[jl * (BT + 1) + il];
        }
    }
}

// The panel path's short-K contractions (K = 128: the panel solve against the
// diagonal block's inverse and the sub-panel updates) on tiles of 64 rows x 128
// columns: twice the workgroups of the 128 x 128 tile for the same rows, so the
// later panels, whose few row tiles leave most CUs idle, finish in about half
// the MFMA time per workgroup.  A workgroup still owns whole 128-column rows of
// C, so the in-place panel solve (C = P) reads its rows before it rewrites them.
// Waves in 2 x 2: rows wi .. wi + 31, columns wj .. wj + 63 (two 32 x 32
// accumulators).  K staged through LDS in double-buffered chunks of 16 by direct
// loads, as in gemm_tile_body.
constexpr int BR = 64;
constexpr int LDS_R64 = 2 * KC * BR + 2 * KC * BT;  // P and Q stages (24 KB)

template <int MODE>
__global__ void __launch_bounds__(NT, 2)
k_gemm_rows64(float *__restrict__ C, int64_t ldc, const float *__restrict__ P, int64_t ldp,
              const float *__restrict__ Q, int64_t ldq, int64_t tilesM, int64_t K, float *__restrict__ CT)
{
    __shared__ float lds[LDS_R64];
    float (*Ps)[KC][BR] = reinterpret_cast<float (*)[KC][BR]>(lds);
    float (*Qs)[KC][BT] = reinterpret_cast<float (*)[KC][BT]>(lds + 2 * KC * BR);
    const int64_t ti = blockIdx.x % tilesM, tj = blockIdx.x / tilesM;
    const int64_t i0 = ti * BR, j0 = tj * BT;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wi = (wave & 1) * 32;
    const int wj = (wave >> 1) * 64;
    const int l32 = lane & 31;
    const int hi = lane >> 5;

    v16f acc[2];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[jb][r] = 0.0f;

    // P stage (64 rows x 16 k): thread t fetches the float4 at row 4 (t % 16),
    // k = t / 16, so wave w fills k-rows 4 w .. 4 w + 3 (1 KB, contiguous);
    // Q stage (128 rows x 16 k) as in gemm_tile_body
    const float *pg = P + (threadIdx.x >> 4) * ldp + i0 + 4 * (threadIdx.x & 15);
    const int lr = 4 * (threadIdx.x & 31);
    const int lp = threadIdx.x >> 5;
    const float *qg0 = Q + lp * ldq + j0 + lr, *qg1 = Q + (lp + 8) * ldq + j0 + lr;
    const int64_t stepP = KC * ldp, stepQ = KC * ldq;
    const int wu = __builtin_amdgcn_readfirstlane(wave);
    auto stage_in = [&](int b) {
        __builtin_amdgcn_global_load_lds((gptr)pg, (lptr)&Ps[b][4 * wu][0], 16, 0, 0);
        __builtin_amdgcn_global_load_lds((gptr)qg0, (lptr)&Qs[b][2 * wu][0], 16, 0, 0);
        __builtin_amdgcn_global_load_lds((gptr)qg1, (lptr)&Qs[b][2 * wu + 8][0], 16, 0, 0);
    };
    stage_in(0);
    __syncthreads();

    const int nst = (int)(K / KC);
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        if (st + 1 < nst) {
            pg += stepP;
            qg0 += stepQ;
            qg1 += stepQ;
            stage_in(buf ^ 1);
        }
#pragma unroll
        for (int kp = 0; kp < KC / 2; ++kp) {
            const int p = 2 * kp + hi;
            const float pv = Ps[buf][p][wi + l32];
            const float q0 = Qs[buf][p][wj + l32];
            const float q1 = Qs[buf][p][wj + 32 + l32];
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(q0, pv, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(q1, pv, acc[1], 0, 0, 0);
        }
        __syncthreads();  // waits for the direct loads of the next stage too
    }

    const int64_t i = i0 + wi + l32;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
        if (MODE == kGemmSub) {
            float cv[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t j = j0 + wj + jb * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
                cv[r] = C[j * ldc + i];
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t j = j0 + wj + jb * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
                C[j * ldc + i] = cv[r] - acc[jb][r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t j = j0 + wj + jb * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
                C[j * ldc + i] = acc[jb][r];
            }
        }
    }
    if (MODE == kGemmSetT) {
        // transposed copy, 64 columns of the tile at a time through LDS (T[jl][il])
        float *T = lds;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            __syncthreads();
            if ((wave >> 1) == half) {
#pragma unroll
                for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int jl = jb * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
                        T[jl * (BR + 1) + wi + l32] = acc[jb][r];
                    }
            }
            __syncthreads();
            const int jl = threadIdx.x & 63;
            for (int il = threadIdx.x >> 6; il < BR; il += NT / 64)
                CT[(i0 + il) * ldc + j0 + half * 64 + jl] = T[jl * (BR + 1) + il];
        }
    }
}

// Trailing symmetric update C -= P P^T on the lower tiles of C only.
// XCD-aware order: workgroups are dealt to the 8 XCDs round-robin by id, so
// id % 8 picks the XCD and consecutive ids of one XCD walk the se x se tiles
// of one super-tile of the lower triangle; the 2 se operand panels of a
// super-tile (2 se x 128 rows x K floats: 4 MB at se = 8, K = 512, or at
// se = 4, K = 1024) stay in that XCD's L2 while its tiles run.
__global__ void __launch_bounds__(NT, 2)
k_syrk_lower(float *__restrict__ C, int64_t ldc, const float *__restrict__ P, int64_t ldp,
             int64_t tilesM, int64_t K, int se)
{
    const int64_t b = blockIdx.x;
    const int64_t xcd = b % kXcds, slot = b / kXcds;
    const int64_t sidx = (slot / (se * se)) * kXcds + xcd, within = slot % (se * se);
    int64_t si, sj;
    tri_index(sidx, si, sj);
    const int64_t ti = si * se + within / se;
    const int64_t tj = sj * se + within % se;
    if (tj > ti || ti >= tilesM) return;  // padding slot (uniform per workgroup)
    gemm_tile_body<kGemmSub, true>(C, ldc, P, ldp, P, ldp, ti, tj, K, nullptr);
}

// Batched factorisation updates at panel offset kk of every active problem.
// Panels are 256 columns wide and go in pairs (kk, kk + 256), as in the
// single-problem factorisation.
//   KIND 0: panel TRSM (SetT) of the 128-column sub-panel at kk, in place
//   KIND 1: update of the next sub-panel's 128 columns by the one at kk
//   KIND 2: trailing SYRK (lower tiles) by the pair of panels at kk (K = 512)
//   KIND 3: strip update of the second panel's columns (every row from
//           kk + 256) by the first panel of the pair at kk (K = 256); the
//           tile above the strip's 128-diagonal is rewritten by the second
//           panel's own TRSM
//   KIND 4: trailing SYRK (lower tiles) by the single panel at kk (K = 256),
//           for the schedule without pairs
template <int KIND>
__global__ void __launch_bounds__(NT, 2)
k_gemm_b(const BProb *__restrict__ Pr, BWork w, int64_t kk)
{
    const int i = bfind(w.pref, w.na, blockIdx.x);
    const BProb &q = Pr[w.plist[i]];
    if (!q.active) return;
    const int64_t u = blockIdx.x - w.pref[i];
    const int64_t np = q.npad;
    float *A = q.A;
    if (KIND == 0) {
        float *A21 = A + kk * np + kk + BT;
        gemm_tile_body<kGemmSetT>(A21, np, A21, np, q.dinv + (kk / BT) * BT * BT, BT, u, 0, BT,
                                  A + (kk + BT) * np + kk);
    } else if (KIND == 1) {
        const float *Pp = A + kk * np + kk + BT;
        gemm_tile_body<kGemmSub>(A + (kk + BT) * np + kk + BT, np, Pp, np, Pp, np, u, 0, BT,
                                 nullptr);
    } else if (KIND == 2) {
        int64_t ti, tj;
        tri_index(u, ti, tj);
        const float *Pp = A + kk * np + kk + 4 * BT;
        gemm_tile_body<kGemmSub, true>(A + (kk + 4 * BT) * np + kk + 4 * BT, np, Pp, np, Pp, np, ti, tj,
                                       4 * BT, nullptr);
    } else if (KIND == 3) {
        const int64_t T = (np - kk - 2 * BT) / BT;
        const float *Pp = A + kk * np + kk + 2 * BT;
        gemm_tile_body<kGemmSub, true>(A + (kk + 2 * BT) * np + kk + 2 * BT, np, Pp, np, Pp, np, u % T, u / T,
                                       2 * BT, nullptr);
    } else {
        int64_t ti, tj;
        tri_index(u, ti, tj);
        const float *Pp = A + kk * np + kk + 2 * BT;
        gemm_tile_body<kGemmSub, true>(A + (kk + 2 * BT) * np + kk + 2 * BT, np, Pp, np, Pp, np, ti, tj,
                                       2 * BT, nullptr);
    }
}

}  // namespace

// work units per problem of the batched updates (see k_gemm_b)
int64_t gemm_b_units(int kind, int64_t npad, int64_t kk)
{
    if (kind == 0 || kind == 1) {
        const int64_t rows = npad - kk - BT;
        return rows > 0 ? rows / BT : 0;
    }
    if (kind == 3) {
        const int64_t rows = npad - kk - 2 * BT;
        return rows > 0 ? 2 * (rows / BT) : 0;
    }
    if (kind == 4) {
        const int64_t rows = npad - kk - 2 * BT;
        const int64_t T = rows > 0 ? rows / BT : 0;
        return T * (T + 1) / 2;
    }
    const int64_t rows = npad - kk - 4 * BT;
    const int64_t T = rows > 0 ? rows / BT : 0;
    return T * (T + 1) / 2;
}

void launch_gemm_b(hipStream_t s, int kind, const BProb *P, const BWork &w, int64_t kk)
{
    if (w.total <= 0) return;
    if (kind == 0)
        hipLaunchKernelGGL(k_gemm_b<0>, dim3((unsigned)w.total), dim3(NT), 0, s, P, w, kk);
    else if (kind == 1)
        hipLaunchKernelGGL(k_gemm_b<1>, dim3((unsigned)w.total), dim3(NT), 0, s, P, w, kk);
    else if (kind == 2)
        hipLaunchKernelGGL(k_gemm_b<2>, dim3((unsigned)w.total), dim3(NT), 0, s, P, w, kk);
    else if (kind == 4)
        hipLaunchKernelGGL(k_gemm_b<4>, dim3((unsigned)w.total), dim3(NT), 0, s, P, w, kk);
    else
        hipLaunchKernelGGL(k_gemm_b<3>, dim3((unsigned)w.total), dim3(NT), 0, s, P, w, kk);
}

void launch_gemm_rows64(hipStream_t s, float *C, int64_t ldc, const float *P, int64_t ldp, const float *Q,
                        int64_t ldq, int64_t M, int64_t N, int64_t K, GemmMode mode, float *CT)
{
    const int64_t tm = M / BR, tn = N / BT;
    if (tm <= 0 || tn <= 0 || K <= 0) return;
    const dim3 g((unsigned)(tm * tn));
    if (mode == kGemmSub)
        hipLaunchKernelGGL(k_gemm_rows64<kGemmSub>, g, dim3(NT), 0, s, C, ldc, P, ldp, Q, ldq, tm, K, CT);
    else if (mode == kGemmSet)
        hipLaunchKernelGGL(k_gemm_rows64<kGemmSet>, g, dim3(NT), 0, s, C, ldc, P, ldp, Q, ldq, tm, K, CT);
    else
        hipLaunchKernelGGL(k_gemm_rows64<kGemmSetT>, g, dim3(NT), 0, s, C, ldc, P, ldp, Q, ldq, tm, K, CT);
}

void launch_syrk_lower(hipStream_t s, float *C, int64_t ldc, const float *P, int64_t ldp,
                       int64_t N, int64_t K)
{
    const int64_t tm = N / BT;
    if (tm <= 0 || K <= 0) return;
    // super-tiles of se x se tiles, in groups of kXcds (one per XCD), sized so
    // their operand panels fit an XCD's 4 MB L2
    const int se = (K > 512) ? 4 : 8;
    const int64_t st = (tm + se - 1) / se;
    const int64_t nsup = st * (st + 1) / 2;
    const int64_t blocks = ((nsup + kXcds - 1) / kXcds) * kXcds * se * se;
    hipLaunchKernelGGL(k_syrk_lower, dim3((unsigned)blocks), dim3(NT), 0, s, C, ldc, P, ldp, tm, K, se);
}

}  // namespace mag
