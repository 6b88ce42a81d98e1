// bctl.hip -- device-side control of the batched solves: the GMRES-based
// iterative refinement and the cutoff search, one thread (or one workgroup)
// per problem, so that a whole step -- choice of each cloud's next scale, tile
// generation, factorisation, refinement to tol, min w, bracket update and the
// Newton derivative -- runs as one captured hipGraph without host decisions.
//
// Every batched kernel skips problems whose descriptor has active == 0.  The
// control kernels keep one flag word per problem (BProb::ints[kIntFlags]) and
// k_gate_b turns a flag into the active bit before each phase, so one launch
// sequence serves problems that take different paths (plain refinement steps,
// GMRES cycles, reverting to the best iterate, finished).
//
// The refinement follows the single solve's rules (api.hip, refine_core):
// x0 = M^{-1} b; each round evaluates r = b - Z x in FP64, keeps the best
// iterate, stops at ||r||_inf <= tol * max(1, ||b||_inf); corrections start as
// plain steps x += M^{-1} r while each gains two digits, then GMRES cycles on
// M^{-1} Z d = M^{-1} r (classical Gram-Schmidt twice, Givens rotations),
// from the best iterate; no progress after a GMRES cycle stops it.
#include "internal.hpp"

#include <cmath>

namespace mag {
namespace {

constexpr int kCtlThreads = 64;
constexpr int LDH = kMaxRestart + 1;  // leading dimension of the stored Hessenberg matrix

inline unsigned blocks_for(int B) { return (unsigned)((B + kCtlThreads - 1) / kCtlThreads); }

__global__ void k_gate_b(BProb *__restrict__ P, int B, int mask)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    P[b].active = ((P[b].ints[kIntFlags] & mask) == mask) ? 1 : 0;
}

__global__ void k_ref_init_b(BProb *__restrict__ P, int B, int64_t bnorm_off, double tol)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    BProb &p = P[b];
    int f = p.ints[kIntFlags];
    f &= ~(F_REF | F_COPYBEST | F_REVERT | F_DOPLAIN | F_DOGMRES | F_INNER | F_LASTPLAIN | F_PLAINMODE |
           F_REVERTED | F_OK);
    if (p.active) {
        double *rc = p.scal + SC_RC;
        f |= F_REF | F_PLAINMODE;
        rc[RC_RNORM] = INFINITY;
        rc[RC_BEST] = INFINITY;
        rc[RC_PREV] = INFINITY;
        rc[RC_TOL] = tol * (bnorm_off >= 0 ? fmax(1.0, p.scal[bnorm_off]) : 1.0);
        rc[RC_INNER] = 0.0;
        rc[RC_ROUND] = 0.0;
    }
    p.ints[kIntFlags] = f;
}

// After the residual of this round (scal[SC_RNORM]) was evaluated for every
// problem with F_REF: keep the best iterate, decide the round's correction.
__global__ void k_ref_decide_b(BProb *__restrict__ P, int B, int final_round, int max_gmres)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    BProb &p = P[b];
    int f = p.ints[kIntFlags] & ~(F_COPYBEST | F_REVERT | F_DOPLAIN | F_DOGMRES | F_INNER);
    if (!(f & F_REF)) {
        p.ints[kIntFlags] = f;
        return;
    }
    double *rc = p.scal + SC_RC;
    const double prev = rc[RC_RNORM];
    const double rnorm = p.scal[SC_RNORM];
    rc[RC_PREV] = prev;
    rc[RC_RNORM] = rnorm;
    const int round = (int)rc[RC_ROUND];
    rc[RC_ROUND] = (double)(round + 1);
    const bool was_reverted = (f & F_REVERTED) != 0;
    f &= ~F_REVERTED;
    if (!(rnorm < rc[RC_BEST]) && !was_reverted) {
        if (!(f & F_LASTPLAIN) || final_round) {
            f &= ~F_REF;  // no progress: the best iterate stands
        } else {
            // the plain step did not help: back to the best iterate, GMRES from there
            f &= ~(F_PLAINMODE | F_LASTPLAIN);
            f |= F_REVERT | F_REVERTED;
        }
        p.ints[kIntFlags] = f;
        return;
    }
    rc[RC_BEST] = rnorm;
    f |= F_COPYBEST;
    if (rnorm <= rc[RC_TOL]) {
        f = (f | F_OK) & ~F_REF;
    } else if (final_round) {
        f &= ~F_REF;
    } else {
        bool stop = false;
        if ((f & F_LASTPLAIN) && rnorm > 1e-2 * prev) f &= ~F_PLAINMODE;
        else if (!(f & F_LASTPLAIN) && !was_reverted && round > 0 && rnorm > 0.5 * prev) stop = true;
        if (rc[RC_INNER] >= (double)max_gmres) stop = true;
        if (stop) {
            f &= ~F_REF;
        } else if (f & F_PLAINMODE) {
            f |= F_DOPLAIN | F_LASTPLAIN;
            rc[RC_INNER] += 1.0;
        } else {
            f |= F_DOGMRES;
            f &= ~F_LASTPLAIN;
        }
    }
    p.ints[kIntFlags] = f;
}

// beta = ||M^{-1} r||_2 in scal[SC_BETA]: a GMRES cycle starts when it is positive
__global__ void k_gmres_start_b(BProb *__restrict__ P, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    BProb &p = P[b];
    int f = p.ints[kIntFlags];
    if (!(f & F_DOGMRES)) return;
    const double beta = p.scal[SC_BETA];
    if (beta > 0.0 && isfinite(beta)) {
        p.scal[SC_RC + RC_BETA] = beta;
        p.scal[SC_RC + RC_KDONE] = 0.0;
        p.scal[SC_G] = beta;
        f |= F_INNER;
    } else {
        f &= ~(F_DOGMRES | F_REF);
    }
    p.ints[kIntFlags] = f;
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One workgroup per problem.  u = V_{k+1} holds M^{-1} Z V_k on entry.
__global__ void __launch_bounds__(256)
k_arnoldi_b(BProb *__restrict__ P, int k, int v0, int kcycle, double inner_tol, int max_gmres)
{
    __shared__ double h[2][kMaxRestart + 1];
    __shared__ double red[4];
    __shared__ double s_hk1;
    BProb &p = P[blockIdx.x];
    if (!(p.ints[kIntFlags] & F_INNER)) return;  // uniform per workgroup
    const int64_t np = p.npad;
    const double *V = p.vec + (int64_t)v0 * np;
    double *u = p.vec + (int64_t)(v0 + k + 1) * np;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = wv; i <= k; i += 4) {
            const double *vi = V + (int64_t)i * np;
            double s = 0.0;
            for (int64_t e = lane; e < np; e += 64) s = fma(vi[e], u[e], s);
            s = wave_sum(s);
            if (lane == 0) h[pass][i] = s;
        }
        __syncthreads();
        for (int64_t e = threadIdx.x; e < np; e += 256) {
            double a = u[e];
            for (int i = 0; i <= k; ++i) a = fma(-h[pass][i], V[(int64_t)i * np + e], a);
            u[e] = a;
        }
        __syncthreads();
    }
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < np; e += 256) s = fma(u[e], u[e], s);
    s = wave_sum(s);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double hk1 = sqrt((red[0] + red[1]) + (red[2] + red[3]));
        double *sc = p.scal;
        double *rc = sc + SC_RC;
        double *Hk = sc + SC_HH + (int64_t)k * LDH;
        double *cs = sc + SC_CS, *sn = sc + SC_SN, *g = sc + SC_G;
        for (int i = 0; i <= k; ++i) Hk[i] = h[0][i] + h[1][i];
        Hk[k + 1] = hk1;
        for (int i = 0; i < k; ++i) {
            const double a = Hk[i], c = Hk[i + 1];
            Hk[i] = cs[i] * a + sn[i] * c;
            Hk[i + 1] = -sn[i] * a + cs[i] * c;
        }
        const double a = Hk[k], c = Hk[k + 1];
        const double rr = hypot(a, c);
        cs[k] = (rr > 0.0) ? a / rr : 1.0;
        sn[k] = (rr > 0.0) ? c / rr : 0.0;
        Hk[k] = rr;
        Hk[k + 1] = 0.0;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        const double inner = rc[RC_INNER] + 1.0;
        rc[RC_INNER] = inner;
        rc[RC_KDONE] = (double)(k + 1);
        const bool cont = fabs(g[k + 1]) > inner_tol * rc[RC_BETA] && hk1 > 0.0 && inner < (double)max_gmres &&
                          k + 1 < kcycle;
        if (!cont) p.ints[kIntFlags] &= ~F_INNER;
        s_hk1 = hk1;
    }
    __syncthreads();
    const double hk1 = s_hk1;
    if (hk1 > 0.0) {
        const double inv = 1.0 / hk1;
        for (int64_t e = threadIdx.x; e < np; e += 256) u[e] = u[e] * inv;
    }
}

// y = H(0:kd, 0:kd)^{-1} g(0:kd) into scal[SC_Y], zero up to kcycle
__global__ void k_gmres_finish_b(BProb *__restrict__ P, int B, int kcycle)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    BProb &p = P[b];
    if (!(p.ints[kIntFlags] & F_DOGMRES)) return;
    const double *sc = p.scal;
    const double *H = sc + SC_HH, *g = sc + SC_G;
    double *y = p.scal + SC_Y;
    const int kd = (int)sc[SC_RC + RC_KDONE];
    for (int a = kd - 1; a >= 0; --a) {
        double acc = g[a];
        for (int j = a + 1; j < kd; ++j) acc -= H[(int64_t)j * LDH + a] * y[j];
        y[a] = acc / H[(int64_t)a * LDH + a];
    }
    for (int j = kd; j < kcycle; ++j) y[j] = 0.0;
}

__global__ void k_axpy_slot_b(BProb *__restrict__ P, int z_slot, int x_slot)
{
    const BProb &q = P[blockIdx.y];
    if (!q.active) return;
    const double *z = q.vec + (int64_t)z_slot * q.npad;
    double *x = q.vec + (int64_t)x_slot * q.npad;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q.npad;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = x[i] + z[i];
}

// ---- cutoff search ------------------------------------------------------------

__global__ void k_search_select_b(BProb *__restrict__ P, SState *__restrict__ S, int B, SParams prm)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    BProb &p = P[b];
    SState &q = S[b];
    int f = p.ints[kIntFlags] & ~(F_SEARCH | F_HI | F_NEEDD | F_BROKEN);
    p.active = 0;
    p.ints[kIntFlags] = f;
    if (q.phase == 2) return;
    if (q.retry) {
        // the FP32 factor broke down at this scale: retake it with a larger diagonal shift
        q.shift = (q.shift == 0.0) ? 1e-6 * fmax(1.0, sqrt((double)p.n)) : q.shift * 10.0;
        if (++q.attempts > 6) {
            q.err = 1;
            q.phase = 2;
            return;
        }
        p.t = q.cur;
        p.shift = q.shift;
        p.active = 1;
        p.ints[kIntFlags] = f | F_SEARCH;
        return;
    }
    q.shift = 0.0;
    q.attempts = 0;
    if (prm.fixed) {
        if (q.phase != 0) return;
        q.cur = p.t;
        p.shift = 0.0;
        p.active = 1;
        p.ints[kIntFlags] = f | F_SEARCH;
        return;
    }
    double tc = 0.0;
    q.cur_newton = 0;
    if (q.phase == 0) {
        // next grid point below the current upper end
        for (;;) {
            if (q.gi < 0) {
                if (q.ext >= prm.max_extend) break;
                ++q.ext;
                q.top *= prm.lo_factor;
                q.gi = prm.grid - 1;
            }
            tc = q.top * pow(prm.lo_factor, (double)(prm.grid - 1 - q.gi) / (prm.grid - 1));
            --q.gi;
            if (!(q.have_hi && tc >= q.hi)) break;
            tc = 0.0;
        }
        if (tc <= 0.0) {
            q.phase = 2;
            q.no_sign = 1;
            return;
        }
    } else {
        if ((q.hi - q.lo) / q.hi <= prm.rtol) {
            q.phase = 2;
            return;
        }
        const double slo = log(q.lo), shi = log(q.hi), mid = 0.5 * (slo + shi);
        double sc = mid;
        q.cur_kind = 0;
        if (prm.ridders) {
            if (q.rid_pending) {
                const double sx = ridders_point(q.ra, q.rga, q.rb, q.rgb, q.rgm);
                if (sx > slo && sx < shi) {
                    sc = sx;
                    q.cur_kind = 2;
                }
            }
            if (q.cur_kind == 0) {
                q.ra = slo;
                q.rga = q.lo_min;
                q.rb = shi;
                q.rgb = q.hi_min;
                q.cur_kind = 1;
            }
        }
        if (prm.newton && q.last_has_d && q.last_d != 0.0) {
            const double sl = log(q.last_t);
            const double sn = sl - q.last_min / (q.last_t * q.last_d);
            const double stp = fabs(sn - sl);
            if (sn > slo && sn < shi && (!q.prev_newton || stp <= 0.5 * q.prev_step)) {
                sc = sn;
                q.cur_newton = 1;
                q.prev_step = stp;
                const double close = 0.25 * prm.rtol;
                if (sc - slo < close) sc = fmin(slo + 0.75 * prm.rtol, mid);
                if (shi - sc < close) sc = fmax(shi - 0.75 * prm.rtol, mid);
            }
        }
        q.prev_newton = q.cur_newton;
        if (!q.cur_newton) q.prev_step = INFINITY;
        tc = exp(sc);
        if (q.cur_kind == 2 && !(tc > q.lo && tc < q.hi)) {
            // the Ridders point rounds onto a bracket end: take the midpoint
            q.ra = slo;
            q.rga = q.lo_min;
            q.rb = shi;
            q.rgb = q.hi_min;
            q.cur_kind = 1;
            tc = exp(mid);
        }
        if (!(tc > q.lo && tc < q.hi)) {
            q.phase = 2;
            return;
        }
    }
    q.cur = tc;
    p.t = tc;
    p.shift = 0.0;
    p.active = 1;
    p.ints[kIntFlags] = f | F_SEARCH;
}

// after the factorisation: a breakdown defers the cloud to the next step (same scale)
__global__ void k_breakdown_b(BProb *__restrict__ P, SState *__restrict__ S, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    BProb &p = P[b];
    int f = p.ints[kIntFlags];
    if (!(f & F_SEARCH)) return;
    if (p.ints[kStBreakdown] != 0) {
        S[b].retry = 1;
        p.active = 0;
        p.ints[kIntFlags] = (f & ~F_SEARCH) | F_BROKEN;
    } else {
        S[b].retry = 0;
    }
}

// min w of this step's solve (scal[SC_SUM + 1]) updates the bracket
__global__ void k_search_update_b(BProb *__restrict__ P, SState *__restrict__ S, int B, SParams prm)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    BProb &p = P[b];
    SState &q = S[b];
    int f = p.ints[kIntFlags];
    if (!(f & F_SEARCH)) return;
    const double mw = p.scal[SC_SUM + 1];
    ++q.solves;
    if (!(f & F_OK)) ++q.unconverged;
    if (prm.fixed) {
        q.phase = 2;
        q.hi_min = mw;
        p.ints[kIntFlags] = f | F_HI;
        return;
    }
    if (q.cur_newton) ++q.newton_steps;
    if (prm.ridders && q.phase == 1) {
        if (q.cur_kind == 2) ++q.newton_steps;
        q.rid_pending = q.cur_kind == 1;
        q.rgm = mw;
    }
    q.last_t = q.cur;
    q.last_min = mw;
    q.last_has_d = 0;
    if (q.phase == 0) {
        if (mw < 0.0) {
            q.have_lo = 1;
            q.lo = q.cur;
            q.lo_min = mw;
            q.phase = 1;
            if (prm.newton) f |= F_NEEDD;
        } else {
            q.have_hi = 1;
            q.hi = q.cur;
            q.hi_min = mw;
            f |= F_HI;
        }
    } else {
        if (mw < 0.0) {
            q.lo = q.cur;
            q.lo_min = mw;
        } else {
            q.hi = q.cur;
            q.hi_min = mw;
            f |= F_HI;
            if (mw < q.eps) q.phase = 2;  // halting rule: 0 <= min w < eps
        }
        if (prm.newton && q.phase == 1) f |= F_NEEDD;
    }
    p.ints[kIntFlags] = f;
}

// d(min w)/dt = (dw/dt)_{argmin} from scal[SC_PICK]
__global__ void k_search_deriv_b(BProb *__restrict__ P, SState *__restrict__ S, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const BProb &p = P[b];
    if (!(p.ints[kIntFlags] & F_NEEDD)) return;
    const double d = p.scal[SC_PICK];
    S[b].last_d = d;
    S[b].last_has_d = isfinite(d) ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_search_count_b(const SState *__restrict__ S, int B, int *out)
{
    __shared__ int cnt[256], err[256];
    int c = 0, e = 0;
    for (int b = threadIdx.x; b < B; b += 256) {
        c += (S[b].phase != 2) ? 1 : 0;
        e |= S[b].err;
    }
    cnt[threadIdx.x] = c;
    err[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            cnt[threadIdx.x] += cnt[threadIdx.x + w];
            err[threadIdx.x] |= err[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = cnt[0];
        out[1] = err[0];
    }
}

}  // namespace

void launch_gate_b(hipStream_t s, BProb *P, int B, int mask)
{
    hipLaunchKernelGGL(k_gate_b, dim3(blocks_for(B)), dim3(kCtlThreads), 0, s, P, B, mask);
}
void launch_ref_init_b(hipStream_t s, BProb *P, int B, int64_t bnorm_off, double tol)
{
    hipLaunchKernelGGL(k_ref_init_b, dim3(blocks_for(B)), dim3(kCtlThreads), 0, s, P, B, bnorm_off, tol);
}
void launch_ref_decide_b(hipStream_t s, BProb *P, int B, int final_round, int max_gmres)
{
    hipLaunchKernelGGL(k_ref_decide_b, dim3(blocks_for(B)), dim3(kCtlThreads), 0, s, P, B, final_round, max_gmres);
}
void launch_gmres_start_b(hipStream_t s, BProb *P, int B)
{
    hipLaunchKernelGGL(k_gmres_start_b, dim3(blocks_for(B)), dim3(kCtlThreads), 0, s, P, B);
}
void launch_arnoldi_b(hipStream_t s, BProb *P, int B, int k, int v0, int kcycle, double inner_tol, int max_gmres)
{
    hipLaunchKernelGGL(k_arnoldi_b, dim3((unsigned)B), dim3(256), 0, s, P, k, v0, kcycle, inner_tol, max_gmres);
}
void launch_gmres_finish_b(hipStream_t s, BProb *P, int B, int kcycle)
{
    hipLaunchKernelGGL(k_gmres_finish_b, dim3(blocks_for(B)), dim3(kCtlThreads), 0, s, P, B, kcycle);
}
void launch_axpy_slot_b(hipStream_t s, BProb *P, int B, int64_t maxpad, int z_slot, int x_slot)
{
    int64_t g = (maxpad + 255) / 256;
    if (g > 64) g = 64;
    hipLaunchKernelGGL(k_axpy_slot_b, dim3((unsigned)g, (unsigned)B), dim3(256), 0, s, P, z_slot, x_slot);
}
void launch_search_select_b(hipStream_t s, BProb *P, SState *S, int B, SParams prm)
{
    hipLaunchKernelGGL(k_search_select_b, dim3(blocks_for(B)), dim3(kCtlThreads), 0, s, P, S, B, prm);
}
void launch_breakdown_b(hipStream_t s, BProb *P, SState *S, int B)
{
    hipLaunchKernelGGL(k_breakdown_b, dim3(blocks_for(B)), dim3(kCtlThreads), 0, s, P, S, B);
}
void launch_search_update_b(hipStream_t s, BProb *P, SState *S, int B, SParams prm)
{
    hipLaunchKernelGGL(k_search_update_b, dim3(blocks_for(B)), dim3(kCtlThreads), 0, s, P, S, B, prm);
}
void launch_search_deriv_b(hipStream_t s, BProb *P, SState *S, int B)
{
    hipLaunchKernelGGL(k_search_deriv_b, dim3(blocks_for(B)), dim3(kCtlThreads), 0, s, P, S, B);
}
void launch_search_count_b(hipStream_t s, const SState *S, int B, int *out)
{
    hipLaunchKernelGGL(k_search_count_b, dim3(1), dim3(256), 0, s, S, B, out);
}

}  // namespace mag
