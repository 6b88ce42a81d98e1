// batch.hip -- many weighting solves of uneven n in one set of launches, and
// the batched cutoff search.
//
// Every phase of the FP32-factor + FP64-refinement solve (tile generation,
// diagonal factor, panel TRSM, sub-panel and trailing updates, triangular
// solves, Z v products, Krylov vector operations) has a batched kernel that
// maps its flat block index through a device work list to (problem, local
// block).  One launch per phase covers every active problem, so a batch of
// small clouds costs about as many launches as one cloud.
//
// The factorisation's launch sequence depends only on the problems' padded
// sizes, so its work lists are uploaded once per batch and the sequence is
// captured in a hipGraph that is replayed for every t-step; the per-step data
// (scale t, active flag, diagonal shift) live in the device descriptor array
// that the kernels read at run time.  The refinement (GMRES) keeps one
// Hessenberg per problem on the host and runs its iterations in lockstep over
// the problems that have not yet converged.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace mag {

namespace {

#define BCHK(x)                                     \
    do {                                            \
        if ((x) != hipSuccess) return MAG_EHIP;     \
    } while (0)
#define BRC(x)                                      \
    do {                                            \
        int rc_ = (x);                              \
        if (rc_ != MAG_OK) return rc_;              \
    } while (0)

// scalar slots of each problem (BProb::scal)
enum : int64_t {
    SC_RNORM = 0,   // ||b - Z x||_inf
    SC_BETA = 1,    // ||M^{-1} r||_2
    SC_SUM = 2,     // sum, min, argmin (3)
    SC_AMAX = 5,
    SC_PICK = 6,    // d(min w)/dt picked at argmin
    SC_H = 16,      // Arnoldi column h (2 (k+1)) and h_{k+1,k}
    SC_Y = 96,      // GMRES solution coefficients
    SC_COUNT = 160
};
constexpr int kIntsPer = 2048;

struct Slots {
    int R, V0, X, Rr, Z, Y, U, Best, Rhs, W, D, DZ, n;
};
Slots slots_for(int restart)
{
    Slots s;
    s.R = restart;
    s.V0 = 0;
    s.X = restart + 1;
    s.Rr = s.X + 1;
    s.Z = s.Rr + 1;
    s.Y = s.Z + 1;
    s.U = s.Y + 1;
    s.Best = s.U + 1;
    s.Rhs = s.Best + 1;
    s.W = s.Rhs + 1;
    s.D = s.W + 1;
    s.DZ = s.D + 1;
    s.n = s.DZ + 1;
    return s;
}

struct Batch {
    mag_ctx *c = nullptr;
    hipStream_t s = nullptr;
    int B = 0, m = 0;
    Slots sl;
    std::vector<BProb> h;  // host copy of the descriptors
    BProb *d = nullptr;    // device descriptors
    int64_t maxpad = 0, maxn = 0;
    // arenas for work lists: persistent (the factorisation schedule) + transient
    char *dev_arena = nullptr, *host_arena = nullptr;
    size_t arena_bytes = 0, persist_used = 0, trans_used = 0;
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_def = nullptr;
    std::vector<double> hostbuf;
    double *dstage = nullptr;  // device staging for gathered scalars

    ~Batch()
    {
        if (graph) hipGraphExecDestroy(graph);
        if (graph_def) hipGraphDestroy(graph_def);
    }

    // Append bytes to an arena region; the host copy is made now, the device
    // copy enqueued on the stream (pinned source).  Transient data are reset at
    // every host sync (all copies done by then).
    template <class T>
    T *put(const std::vector<T> &v, bool persist)
    {
        const size_t bytes = ((v.size() * sizeof(T)) + 255) / 256 * 256;
        size_t &used = persist ? persist_used : trans_used;
        const size_t base = persist ? 0 : arena_bytes / 2;
        if (base + used + bytes > (persist ? arena_bytes / 2 : arena_bytes)) return nullptr;
        char *hp = host_arena + base + used;
        char *dp = dev_arena + base + used;
        if (!v.empty()) {
            std::memcpy(hp, v.data(), v.size() * sizeof(T));
            if (hipMemcpyAsync(dp, hp, v.size() * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess)
                return nullptr;
        }
        used += bytes;
        return reinterpret_cast<T *>(dp);
    }
    void reset_transient() { trans_used = 0; }

    // Work list over problem ids `ids` with `units(p)` work units each.
    template <class F>
    int make_work(const std::vector<int> &ids, F units, bool persist, BWork &w)
    {
        std::vector<int> pl;
        std::vector<int64_t> pref(1, 0);
        for (int p : ids) {
            const int64_t u = units(p);
            if (u <= 0) continue;
            pl.push_back(p);
            pref.push_back(pref.back() + u);
        }
        w.na = (int)pl.size();
        w.total = pref.back();
        if (w.na == 0) {
            w.plist = nullptr;
            w.pref = nullptr;
            return MAG_OK;
        }
        w.plist = put(pl, persist);
        w.pref = put(pref, persist);
        return (w.plist && w.pref) ? MAG_OK : MAG_ENOMEM;
    }

    int upload_desc() { return hipMemcpyAsync(d, h.data(), sizeof(BProb) * B, hipMemcpyHostToDevice, s) == hipSuccess ? MAG_OK : MAG_EHIP; }

    int sync()
    {
        BCHK(hipStreamSynchronize(s));
        reset_transient();
        return MAG_OK;
    }

    // gather `cnt` scalars at `off` of the listed problems to the host
    int gather(const int *plist_dev, int na, int64_t off, int cnt, std::vector<double> &out)
    {
        out.resize((size_t)na * cnt);
        if (na == 0) return MAG_OK;
        launch_gather_scal_b(s, d, plist_dev, na, off, cnt, dstage);
        BCHK(hipMemcpyAsync(out.data(), dstage, sizeof(double) * na * cnt, hipMemcpyDeviceToHost, s));
        return sync();
    }
};

// Allocate every problem's buffers and the descriptors.  items: (X, n, t).
int batch_setup(mag_ctx *c, Batch &bt, const std::vector<const double *> &Xs,
                const std::vector<int64_t> &ns, int m, const std::vector<double> &ts, int restart)
{
    bt.c = c;
    bt.s = c->stream;
    bt.B = (int)ns.size();
    bt.m = m;
    bt.sl = slots_for(restart);
    const int B = bt.B;
    size_t fac = 0, dv = 0, vec = 0, part = 0;
    std::vector<int64_t> np(B);
    for (int b = 0; b < B; ++b) {
        np[b] = round_up(ns[b], kPad);
        fac += (size_t)np[b] * np[b];
        dv += (size_t)np[b] * kTile;
        vec += (size_t)bt.sl.n * np[b];
        part += std::max(std::max(zmv_partial_doubles(ns[b]), pair_partial_doubles(ns[b], 1)),
                         blas1_partial_doubles(restart + 2)) + 64;
        bt.maxpad = std::max(bt.maxpad, np[b]);
        bt.maxn = std::max(bt.maxn, ns[b]);
    }
    BRC(ensure(c, c->bfactor, sizeof(float) * fac));
    BRC(ensure(c, c->bdinv, sizeof(float) * dv));
    BRC(ensure(c, c->bvec, sizeof(double) * vec));
    BRC(ensure(c, c->bscal, sizeof(double) * (size_t)B * SC_COUNT));
    BRC(ensure(c, c->bpartial, sizeof(double) * part));
    BRC(ensure(c, c->bints, sizeof(int) * (size_t)B * kIntsPer));
    BRC(ensure(c, c->bdesc, sizeof(BProb) * B));
    BRC(ensure(c, c->bstage, sizeof(double) * ((size_t)B * 128 + 64)));
    // work-list arena: generous for the schedule (~6 launches per 128 columns)
    const size_t arena = std::max<size_t>((size_t)1 << 22, (size_t)B * (bt.maxpad / 128 + 4) * 8 * 256);
    BRC(ensure(c, c->barena, arena));
    if (c->bhost_bytes < arena) {
        if (c->bhost) hipHostFree(c->bhost);
        c->bhost = nullptr;
        c->bhost_bytes = 0;
        if (hipHostMalloc(&c->bhost, arena, hipHostMallocDefault) != hipSuccess) return MAG_ENOMEM;
        c->bhost_bytes = arena;
    }
    bt.dev_arena = (char *)c->barena.p;
    bt.host_arena = (char *)c->bhost;
    bt.arena_bytes = arena;
    bt.d = (BProb *)c->bdesc.p;
    bt.dstage = (double *)c->bstage.p;
    bt.h.resize(B);
    float *fp = (float *)c->bfactor.p;
    float *dp = (float *)c->bdinv.p;
    double *vp = (double *)c->bvec.p;
    double *pp = (double *)c->bpartial.p;
    for (int b = 0; b < B; ++b) {
        BProb &q = bt.h[b];
        q.X = Xs[b];
        q.n = ns[b];
        q.npad = np[b];
        q.t = ts[b];
        q.shift = 0.0;
        q.A = fp;
        fp += (size_t)np[b] * np[b];
        q.dinv = dp;
        dp += (size_t)np[b] * kTile;
        q.vec = vp;
        vp += (size_t)bt.sl.n * np[b];
        q.scal = (double *)c->bscal.p + (size_t)b * SC_COUNT;
        q.partial = pp;
        pp += std::max(std::max(zmv_partial_doubles(ns[b]), pair_partial_doubles(ns[b], 1)),
                       blas1_partial_doubles(restart + 2)) + 64;
        q.ints = (int *)c->bints.p + (size_t)b * kIntsPer;
        q.m = m;
        q.active = 1;
    }
    BCHK(hipMemsetAsync(c->bvec.p, 0, sizeof(double) * vec, bt.s));
    return bt.upload_desc();
}

// Record the factorisation schedule of all problems into a hipGraph.
int batch_build_graph(Batch &bt)
{
    std::vector<int> all(bt.B);
    for (int b = 0; b < bt.B; ++b) all[b] = b;
    // work lists (persistent arena), built before capture
    struct Launch {
        int kind;  // 0 trsm, 1 subupdate, 2 syrk, 3 potrf, 4 tilegen, 5 zero status, 6 strip
        int64_t kk;
        BWork w;
    };
    std::vector<Launch> seq;
    BWork wall;
    BRC(bt.make_work(all, [&](int) { return (int64_t)1; }, true, wall));
    seq.push_back({5, 0, wall});
    BWork wt;
    BRC(bt.make_work(all, [&](int p) { return tilegen32_blocks(bt.h[p].npad); }, true, wt));
    seq.push_back({4, 0, wt});
    // panels of kPanel columns in pairs: first panel, strip update of the second
    // panel by the first, second panel, then one trailing update by both
    for (int64_t k = 0; k < bt.maxpad; k += 2 * kPanel) {
        for (int half = 0; half < 2; ++half) {
            const int64_t kp = k + half * kPanel;
            if (half == 1) {
                BWork ws;
                BRC(bt.make_work(all, [&](int p) { return kp < bt.h[p].npad ? gemm_b_units(3, bt.h[p].npad, k) : 0; }, true, ws));
                seq.push_back({6, k, ws});
            }
            for (int sub = 0; sub < kPanel / kTile; ++sub) {
                const int64_t kk = kp + sub * kTile;
                BWork wp;
                BRC(bt.make_work(all, [&](int p) { return (int64_t)(kk < bt.h[p].npad ? 1 : 0); }, true, wp));
                seq.push_back({3, kk, wp});
                BWork w0;
                BRC(bt.make_work(all, [&](int p) { return kk < bt.h[p].npad ? gemm_b_units(0, bt.h[p].npad, kk) : 0; }, true, w0));
                seq.push_back({0, kk, w0});
                if (sub == 0) {
                    BWork w1;
                    BRC(bt.make_work(all, [&](int p) { return kk < bt.h[p].npad ? gemm_b_units(1, bt.h[p].npad, kk) : 0; }, true, w1));
                    seq.push_back({1, kk, w1});
                }
            }
        }
        BWork w2;
        BRC(bt.make_work(all, [&](int p) { return k < bt.h[p].npad ? gemm_b_units(2, bt.h[p].npad, k) : 0; }, true, w2));
        seq.push_back({2, k, w2});
    }
    BCHK(hipStreamSynchronize(bt.s));  // schedule uploaded
    BCHK(hipStreamBeginCapture(bt.s, hipStreamCaptureModeThreadLocal));
    for (const Launch &L : seq) {
        switch (L.kind) {
        case 5: launch_zero_status_b(bt.s, bt.d, L.w.plist, L.w.na); break;
        case 4: launch_tilegen32_b(bt.s, bt.d, L.w); break;
        case 3: launch_potrf128_b(bt.s, bt.d, L.w, L.kk); break;
        case 6: launch_gemm_b(bt.s, 3, bt.d, L.w, L.kk); break;
        default: launch_gemm_b(bt.s, L.kind, bt.d, L.w, L.kk); break;
        }
    }
    if (hipStreamEndCapture(bt.s, &bt.graph_def) != hipSuccess) return MAG_EHIP;
    BCHK(hipGraphInstantiate(&bt.graph, bt.graph_def, nullptr, nullptr, 0));
    return MAG_OK;
}

// Factor every active problem (graph replay), retrying problems whose FP32
// factor broke down with a growing diagonal shift.
int batch_factor(Batch &bt, std::vector<int> &shifted)
{
    shifted.assign(bt.B, 0);
    std::vector<int> saved_active(bt.B);
    for (int b = 0; b < bt.B; ++b) saved_active[b] = bt.h[b].active;
    for (int attempt = 0;; ++attempt) {
        BRC(bt.upload_desc());
        BCHK(hipGraphLaunch(bt.graph, bt.s));
        // breakdown status of every problem
        std::vector<int> st(bt.B, 0);
        for (int b = 0; b < bt.B; ++b)
            if (bt.h[b].active)
                BCHK(hipMemcpyAsync(&st[b], bt.h[b].ints + kStBreakdown, sizeof(int), hipMemcpyDeviceToHost, bt.s));
        BRC(bt.sync());
        bool any = false;
        for (int b = 0; b < bt.B; ++b) {
            if (bt.h[b].active && st[b] != 0) {
                any = true;
                shifted[b] = 1;
                const double n = (double)bt.h[b].n;
                bt.h[b].shift = bt.h[b].shift == 0.0 ? 1e-6 * std::max(1.0, std::sqrt(n)) : bt.h[b].shift * 10.0;
            } else {
                bt.h[b].active = 0;  // factor done: not refactored in the next attempt
            }
        }
        if (!any) break;
        if (attempt >= 6) return MAG_ENOTPD;
    }
    for (int b = 0; b < bt.B; ++b) bt.h[b].active = saved_active[b];
    return bt.upload_desc();
}

struct BRefine {
    double best = INFINITY, rnorm = INFINITY, prev = INFINITY, tol = 1e-12;
    int outer = 0, inner = 0, done = 0, ok = 0;
    int plain = 1, last_plain = 0, reverted = 0;  // plain refinement steps first (see refine_core)
    std::vector<double> H, cs, sn, g;
    int kdone = 0, inner_done = 0;
    double beta = 0.0;
};

// GMRES-based iterative refinement for Z x = b of every problem in `ids`
// (b = slot rhs_slot, zero padded); the best iterate lands in slot Best.
int batch_refine(Batch &bt, const std::vector<int> &ids, int rhs_slot, const std::vector<double> &bnorm,
                 const mag_opts &o, std::vector<BRefine> &st)
{
    const Slots &S = bt.sl;
    const int R = S.R;
    const double tol = o.tol > 0 ? o.tol : 1e-12;
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-10;
    const int max_gmres = o.max_gmres > 0 ? o.max_gmres : 200;
    st.assign(bt.B, BRefine());
    for (int p : ids) {
        st[p].tol = tol * std::max(1.0, bnorm[p]);
        st[p].H.assign((size_t)(R + 1) * R, 0.0);
        st[p].cs.assign(R, 0.0);
        st[p].sn.assign(R, 0.0);
        st[p].g.assign(R + 1, 0.0);
    }
    auto prec_units = [&](int p) { return prec_b_units(bt.h[p].npad); };
    auto zmv_units = [&](int p) { return zmv_b_units(bt.h[p].n, bt.m); };
    auto red_units = [&](int p) { return zmv_b_reduce_units(bt.h[p].n, bt.m); };
    auto one = [&](int) { return (int64_t)1; };

    // x0 = M^{-1} b
    {
        BWork wp;
        BRC(bt.make_work(ids, prec_units, false, wp));
        launch_prec_apply_b(bt.s, bt.d, wp, rhs_slot, S.Y, S.X);
    }
    std::vector<double> hv;
    for (int outer = 0; outer < std::max(1, o.max_outer); ++outer) {
        std::vector<int> L;
        for (int p : ids)
            if (!st[p].done) L.push_back(p);
        if (L.empty()) break;
        BWork wz, wr, w1;
        BRC(bt.make_work(L, zmv_units, false, wz));
        BRC(bt.make_work(L, red_units, false, wr));
        BRC(bt.make_work(L, one, false, w1));
        launch_zmv_b(bt.s, bt.m, bt.d, wz, wr, S.X, S.Rr, rhs_slot, 1, SC_RNORM);
        BRC(bt.gather(w1.plist, w1.na, SC_RNORM, 1, hv));
        std::vector<int> G;        // problems that improved (>= 0: and take a correction)
        std::vector<int> revert;   // plain step without progress: back to the best iterate
        for (size_t i = 0; i < L.size(); ++i) {
            const int p = L[i];
            BRefine &r = st[p];
            r.prev = r.rnorm;
            r.rnorm = hv[i];
            r.outer = outer + 1;
            const int was_reverted = r.reverted;
            r.reverted = 0;
            // after a revert x is the best iterate again: its residual equals the best one
            if (!(r.rnorm < r.best) && !was_reverted) {
                if (!r.last_plain) {
                    r.done = 1;
                    continue;
                }
                // the residual is recomputed from the best iterate next outer step
                r.plain = r.last_plain = 0;
                r.reverted = 1;
                revert.push_back(p);
                continue;
            }
            r.best = r.rnorm;
            if (r.rnorm <= r.tol) {
                r.done = 1;
                r.ok = 1;
                G.push_back(-1 - p);  // mark: copy x to best, no correction
                continue;
            }
            if (r.last_plain && r.rnorm > 1e-2 * r.prev) r.plain = 0;
            else if (!r.last_plain && !was_reverted && outer > 0 && r.rnorm > 0.5 * r.prev) {
                r.done = 1;  // stagnation
                G.push_back(-1 - p);
                continue;
            }
            if (r.inner >= max_gmres) {
                r.done = 1;
                G.push_back(-1 - p);
                continue;
            }
            G.push_back(p);
        }
        // keep the best iterate of every problem that improved
        std::vector<int> improved, run, plain;
        for (int g : G) {
            improved.push_back(g < 0 ? -1 - g : g);
            if (g >= 0) (st[g].plain ? plain : run).push_back(g);
        }
        if (!improved.empty()) {
            BWork wi;
            BRC(bt.make_work(improved, one, false, wi));
            launch_copy_b(bt.s, bt.d, wi.plist, wi.na, bt.maxpad, S.X, S.Best);
        }
        if (!revert.empty()) {
            BWork wv;
            BRC(bt.make_work(revert, one, false, wv));
            launch_copy_b(bt.s, bt.d, wv.plist, wv.na, bt.maxpad, S.Best, S.X);
        }
        if (!plain.empty()) {
            // x += M^{-1} r
            BWork pp, p1;
            BRC(bt.make_work(plain, prec_units, false, pp));
            BRC(bt.make_work(plain, one, false, p1));
            launch_prec_apply_b(bt.s, bt.d, pp, S.Rr, S.Y, S.Z);
            const double *ones = bt.put(std::vector<double>(plain.size(), 1.0), false);
            if (!ones) return MAG_ENOMEM;
            launch_multi_axpy_hb(bt.s, bt.d, p1.plist, p1.na, bt.maxpad, S.Z, 1, ones, S.X, 1.0);
            for (int p : plain) {
                ++st[p].inner;
                st[p].last_plain = 1;
            }
        }
        for (int p : run) st[p].last_plain = 0;
        if (run.empty()) continue;
        BWork gp, g1;
        BRC(bt.make_work(run, prec_units, false, gp));
        BRC(bt.make_work(run, one, false, g1));
        launch_prec_apply_b(bt.s, bt.d, gp, S.Rr, S.Y, S.Z);
        launch_nrm2_b(bt.s, bt.d, g1.plist, g1.na, S.Z, SC_BETA);
        BRC(bt.gather(g1.plist, g1.na, SC_BETA, 1, hv));
        std::vector<int> act;
        for (size_t i = 0; i < run.size(); ++i) {
            const int p = run[i];
            BRefine &r = st[p];
            r.beta = hv[i];
            std::fill(r.H.begin(), r.H.end(), 0.0);
            std::fill(r.g.begin(), r.g.end(), 0.0);
            r.g[0] = r.beta;
            r.kdone = 0;
            r.inner_done = 0;
            if (r.beta > 0.0 && std::isfinite(r.beta)) act.push_back(p);
            else r.done = 1;
        }
        if (act.empty()) continue;
        {
            BWork a1;
            BRC(bt.make_work(act, one, false, a1));
            launch_scale_inv_b(bt.s, bt.d, a1.plist, a1.na, bt.maxpad, S.Z, S.V0, SC_BETA);
        }
        std::vector<int> run2 = act;
        for (int k = 0; k < R && !act.empty(); ++k) {
            BWork az, ar, ap, a1;
            BRC(bt.make_work(act, zmv_units, false, az));
            BRC(bt.make_work(act, red_units, false, ar));
            BRC(bt.make_work(act, prec_units, false, ap));
            BRC(bt.make_work(act, one, false, a1));
            launch_zmv_b(bt.s, bt.m, bt.d, az, ar, S.V0 + k, S.U, -1, 0, 0);
            launch_prec_apply_b(bt.s, bt.d, ap, S.U, S.Y, S.V0 + k + 1);
            launch_multidot_b(bt.s, bt.d, a1.plist, a1.na, S.V0, k + 1, S.V0 + k + 1, SC_H);
            launch_multi_axpy_b(bt.s, bt.d, a1.plist, a1.na, bt.maxpad, S.V0, k + 1, SC_H, S.V0 + k + 1, -1.0);
            launch_multidot_b(bt.s, bt.d, a1.plist, a1.na, S.V0, k + 1, S.V0 + k + 1, SC_H + k + 1);
            launch_multi_axpy_b(bt.s, bt.d, a1.plist, a1.na, bt.maxpad, S.V0, k + 1, SC_H + k + 1, S.V0 + k + 1, -1.0);
            launch_nrm2_b(bt.s, bt.d, a1.plist, a1.na, S.V0 + k + 1, SC_H + 2 * (k + 1));
            const int cnt = 2 * (k + 1) + 1;
            BRC(bt.gather(a1.plist, a1.na, SC_H, cnt, hv));
            std::vector<int> next, scale;
            for (size_t i = 0; i < act.size(); ++i) {
                const int p = act[i];
                BRefine &r = st[p];
                const double *hb = hv.data() + i * cnt;
                const double hk1 = hb[2 * (k + 1)];
                double *Hk = r.H.data() + (size_t)k * (R + 1);
                for (int q = 0; q <= k; ++q) Hk[q] = hb[q] + hb[k + 1 + q];
                Hk[k + 1] = hk1;
                for (int q = 0; q < k; ++q) {
                    const double a = Hk[q], b2 = Hk[q + 1];
                    Hk[q] = r.cs[q] * a + r.sn[q] * b2;
                    Hk[q + 1] = -r.sn[q] * a + r.cs[q] * b2;
                }
                const double a = Hk[k], b2 = Hk[k + 1];
                const double rr = std::hypot(a, b2);
                r.cs[k] = rr > 0 ? a / rr : 1.0;
                r.sn[k] = rr > 0 ? b2 / rr : 0.0;
                Hk[k] = rr;
                Hk[k + 1] = 0.0;
                r.g[k + 1] = -r.sn[k] * r.g[k];
                r.g[k] = r.cs[k] * r.g[k];
                ++r.inner;
                r.kdone = k + 1;
                if (hk1 > 0.0) scale.push_back(p);
                if (std::fabs(r.g[k + 1]) > inner_tol * r.beta && hk1 > 0.0 && r.inner < max_gmres)
                    next.push_back(p);
            }
            if (!scale.empty()) {
                BWork s1;
                BRC(bt.make_work(scale, one, false, s1));
                launch_scale_inv_b(bt.s, bt.d, s1.plist, s1.na, bt.maxpad, S.V0 + k + 1, S.V0 + k + 1,
                                   SC_H + 2 * (k + 1));
            }
            act.swap(next);
        }
        // x += V y: coefficients of all problems in one array (zero padded to the
        // largest Krylov dimension; unused basis slots hold finite values)
        int kmax = 0;
        for (int p : run2) kmax = std::max(kmax, st[p].kdone);
        if (kmax > 0) {
            std::vector<double> Y((size_t)run2.size() * kmax, 0.0);
            for (size_t i = 0; i < run2.size(); ++i) {
                BRefine &r = st[run2[i]];
                double *y = Y.data() + i * kmax;
                for (int a = r.kdone - 1; a >= 0; --a) {
                    double acc = r.g[a];
                    for (int j = a + 1; j < r.kdone; ++j) acc -= r.H[(size_t)j * (R + 1) + a] * y[j];
                    y[a] = acc / r.H[(size_t)a * (R + 1) + a];
                }
            }
            const double *Yd = bt.put(Y, false);
            BWork wy;
            BRC(bt.make_work(run2, one, false, wy));
            if (!Yd) return MAG_ENOMEM;
            launch_multi_axpy_hb(bt.s, bt.d, wy.plist, wy.na, bt.maxpad, S.V0, kmax, Yd, S.X, 1.0);
        }
    }
    return MAG_OK;
}

int validate_batch(mag_ctx *c, const std::vector<const double *> &Xs, const std::vector<int64_t> &ns,
                   int m)
{
    for (size_t b = 0; b < ns.size(); ++b) {
        if (ns[b] < 1) return MAG_EINVAL;
        BRC(check_points(c, Xs[b], ns[b], m));
    }
    return MAG_OK;
}

}  // namespace
}  // namespace mag

using namespace mag;

extern "C" {

int mag_weighting_batch(mag_ctx *c, int32_t B, const double *X, const int64_t *offs, int32_t m,
                        const double *t, double *w, double *M, const mag_opts *opts, mag_info *info)
{
    if (!c || B < 1 || !X || !offs || !t || !w || m < 1) return MAG_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return MAG_EHIP;
    mag_opts o;
    if (opts) o = *opts;
    else mag_opts_default(&o);
    std::vector<const double *> Xs(B);
    std::vector<int64_t> ns(B);
    std::vector<double> ts(B);
    for (int b = 0; b < B; ++b) {
        if (offs[b + 1] < offs[b] || !(std::isfinite(t[b]) && t[b] > 0.0)) return MAG_EINVAL;
        Xs[b] = X + offs[b] * m;
        ns[b] = offs[b + 1] - offs[b];
        ts[b] = t[b];
    }
    BRC(validate_batch(c, Xs, ns, m));
    Batch bt;
    const int restart = std::min(38, std::max(1, o.gmres_restart));
    BRC(batch_setup(c, bt, Xs, ns, m, ts, restart));
    BRC(batch_build_graph(bt));
    std::vector<int> shifted;
    BRC(batch_factor(bt, shifted));
    std::vector<int> ids(B);
    for (int b = 0; b < B; ++b) ids[b] = b;
    {
        BWork w1;
        BRC(bt.make_work(ids, [](int) { return (int64_t)1; }, false, w1));
        launch_fill_b(bt.s, bt.d, w1.plist, w1.na, bt.maxpad, bt.sl.Rhs, 1.0, true);
    }
    std::vector<BRefine> st;
    std::vector<double> bn(B, 1.0);
    BRC(batch_refine(bt, ids, bt.sl.Rhs, bn, o, st));
    BWork w1;
    BRC(bt.make_work(ids, [](int) { return (int64_t)1; }, false, w1));
    std::vector<int64_t> po(B);
    for (int b = 0; b < B; ++b) po[b] = offs[b] - offs[0];
    const int64_t *po_dev = bt.put(po, false);
    if (!po_dev) return MAG_ENOMEM;
    launch_unpack_b(bt.s, bt.d, w1.plist, w1.na, po_dev, bt.sl.Best, w, bt.maxn);
    launch_summin_b(bt.s, bt.d, w1.plist, w1.na, bt.sl.Best, SC_SUM);
    std::vector<double> sums;
    BRC(bt.gather(w1.plist, w1.na, SC_SUM, 3, sums));
    int rc = MAG_OK;
    for (int b = 0; b < B; ++b) {
        if (M) M[b] = sums[3 * b];
        if (!st[b].ok) rc = MAG_ENOCONV;
        if (info) {
            mag_info &f = info[b];
            std::memset(&f, 0, sizeof(f));
            f.status = st[b].ok ? MAG_OK : MAG_ENOCONV;
            f.outer_iters = st[b].outer;
            f.gmres_iters = st[b].inner;
            f.shifted = shifted[b];
            f.shift = bt.h[b].shift;
            f.resid_inf = st[b].best;
            f.magnitude = sums[3 * b];
            f.min_w = sums[3 * b + 1];
            f.argmin_w = (int64_t)sums[3 * b + 2];
        }
    }
    return rc;
}

// ---- batched cutoff search -----------------------------------------------------

int mag_tplus_batch(mag_ctx *c, int32_t B, const double *X, const int64_t *offs, int32_t m,
                    const mag_tplus_opts *topts, const mag_opts *sopts, double *t_plus, double *w,
                    mag_tplus_info *info)
{
    if (!c || B < 1 || !X || !offs || !t_plus || m < 1) return MAG_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return MAG_EHIP;
    mag_tplus_opts to;
    if (topts) to = *topts;
    else mag_tplus_opts_default(&to);
    mag_opts o;
    if (sopts) o = *sopts;
    else mag_opts_default(&o);
    if (to.grid < 2 || !(to.lo_factor > 0.0 && to.lo_factor < 1.0) || !(to.rtol > 0.0)) return MAG_EINVAL;
    if (to.method != MAG_TPLUS_BISECT && to.method != MAG_TPLUS_RIDDERS) return MAG_EINVAL;
    std::vector<const double *> Xs(B);
    std::vector<int64_t> ns(B);
    for (int b = 0; b < B; ++b) {
        if (offs[b + 1] < offs[b]) return MAG_EINVAL;
        Xs[b] = X + offs[b] * m;
        ns[b] = offs[b + 1] - offs[b];
    }
    BRC(validate_batch(c, Xs, ns, m));
    if (m > pair_max_dim() && to.newton) to.newton = 0;
    const bool ridders = to.method == MAG_TPLUS_RIDDERS;
    if (ridders) to.newton = 0;

    // per-cloud state of the search (same rules as mag_tplus)
    struct Cloud {
        int phase = 0;  // 0 grid scan, 1 bracket refinement, 2 done
        double tb = 0, dmin = 0, eps = 0, top = 0;
        int gi = 0, ext = 0;
        bool have_hi = false, have_lo = false, prev_newton = false, want_deriv = false;
        double hi = 0, hi_min = 0, lo = 0, lo_min = 0;
        double last_t = 0, last_min = 0, last_d = 0;
        bool last_has_d = false;
        double prev_step = INFINITY;
        int solves = 0, newton_steps = 0, no_sign = 0;
        double cur = 0;
        bool cur_newton = false;
        // Ridders: the bracket (log t, min w) at the start of a step, whether its
        // midpoint has been evaluated (then the Ridders point is next), and what
        // the current evaluation is (0 other, 1 midpoint, 2 Ridders point)
        double ra = 0, rga = 0, rb = 0, rgb = 0, rgm = 0;
        bool rid_pending = false;
        int cur_kind = 0;
    };
    std::vector<Cloud> cl(B);
    std::vector<double> ts(B, 1.0);
    for (int b = 0; b < B; ++b) {
        Cloud &q = cl[b];
        if (ns[b] <= 2) {
            q.phase = 2;
            q.no_sign = 1;
            continue;
        }
        double dm = 0.0;
        BRC(mag_dmin(c, Xs[b], ns[b], m, &dm));
        q.dmin = dm;
        q.tb = std::log((double)(ns[b] - 1)) / dm;
        q.eps = to.eps > 0.0 ? to.eps : (double)ns[b] * std::ldexp(1.0, -53);
        q.top = q.tb;
        q.gi = to.grid - 1;
        ts[b] = q.tb;
    }
    Batch bt;
    const int restart = std::min(38, std::max(1, o.gmres_restart));
    BRC(batch_setup(c, bt, Xs, ns, m, ts, restart));
    BRC(batch_build_graph(bt));
    const Slots &S = bt.sl;
    auto one = [](int) { return (int64_t)1; };
    const bool newton = to.newton != 0;

    for (int step = 0; step < 1000; ++step) {
        // choose every active cloud's next scale
        std::vector<int> act;
        for (int b = 0; b < B; ++b) {
            Cloud &q = cl[b];
            bt.h[b].active = 0;
            if (q.phase == 2) continue;
            double tc = 0.0;
            q.cur_newton = false;
            if (q.phase == 0) {
                // next grid point below the current upper end
                for (;;) {
                    if (q.gi < 0) {
                        if (q.ext >= to.max_extend) break;
                        ++q.ext;
                        q.top *= to.lo_factor;
                        q.gi = to.grid - 1;
                    }
                    tc = q.top * std::pow(to.lo_factor, (double)(to.grid - 1 - q.gi) / (to.grid - 1));
                    --q.gi;
                    if (!(q.have_hi && tc >= q.hi)) break;
                    tc = 0.0;
                }
                if (tc <= 0.0) {
                    q.phase = 2;
                    q.no_sign = 1;
                    continue;
                }
            } else {
                if ((q.hi - q.lo) / q.hi <= to.rtol) {
                    q.phase = 2;
                    continue;
                }
                const double slo = std::log(q.lo), shi = std::log(q.hi), mid = 0.5 * (slo + shi);
                double sc = mid;
                q.cur_kind = 0;
                if (ridders) {
                    // the same steps as mag_tplus, one evaluation per batched solve
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
                if (newton && q.last_has_d && q.last_d != 0.0) {
                    const double sl = std::log(q.last_t);
                    const double sn = sl - q.last_min / (q.last_t * q.last_d);
                    const double stp = std::fabs(sn - sl);
                    if (sn > slo && sn < shi && (!q.prev_newton || stp <= 0.5 * q.prev_step)) {
                        sc = sn;
                        q.cur_newton = true;
                        q.prev_step = stp;
                        const double close = 0.25 * to.rtol;
                        if (sc - slo < close) sc = std::min(slo + 0.75 * to.rtol, mid);
                        if (shi - sc < close) sc = std::max(shi - 0.75 * to.rtol, mid);
                    }
                }
                q.prev_newton = q.cur_newton;
                if (!q.cur_newton) q.prev_step = INFINITY;
                tc = std::exp(sc);
                if (q.cur_kind == 2 && !(tc > q.lo && tc < q.hi)) {
                    // the Ridders point rounds onto a bracket end: take the midpoint
                    q.ra = slo;
                    q.rga = q.lo_min;
                    q.rb = shi;
                    q.rgb = q.hi_min;
                    q.cur_kind = 1;
                    tc = std::exp(mid);
                }
                if (!(tc > q.lo && tc < q.hi)) {
                    q.phase = 2;
                    continue;
                }
            }
            q.cur = tc;
            bt.h[b].t = tc;
            bt.h[b].active = 1;
            bt.h[b].shift = 0.0;
            act.push_back(b);
        }
        if (act.empty()) break;
        // one batched solve at every active cloud's scale
        std::vector<int> shifted;
        BRC(batch_factor(bt, shifted));
        {
            BWork w1;
            BRC(bt.make_work(act, one, false, w1));
            launch_fill_b(bt.s, bt.d, w1.plist, w1.na, bt.maxpad, S.Rhs, 1.0, true);
        }
        std::vector<BRefine> st;
        std::vector<double> bn(B, 1.0);
        BRC(batch_refine(bt, act, S.Rhs, bn, o, st));
        std::vector<double> mins;
        {
            BWork w1;
            BRC(bt.make_work(act, one, false, w1));
            launch_summin_b(bt.s, bt.d, w1.plist, w1.na, S.Best, SC_SUM);
            launch_copy_b(bt.s, bt.d, w1.plist, w1.na, bt.maxpad, S.Best, S.DZ);  // w of this step
            BRC(bt.gather(w1.plist, w1.na, SC_SUM, 3, mins));
        }
        // update the states; collect clouds that need d(min w)/dt at this point
        std::vector<int> need_d;
        for (size_t i = 0; i < act.size(); ++i) {
            const int b = act[i];
            Cloud &q = cl[b];
            const double mw = mins[3 * i + 1];
            ++q.solves;
            if (q.cur_newton) ++q.newton_steps;
            if (ridders && q.phase == 1) {
                if (q.cur_kind == 2) ++q.newton_steps;
                q.rid_pending = q.cur_kind == 1;
                q.rgm = mw;
            }
            q.last_t = q.cur;
            q.last_min = mw;
            q.last_has_d = false;
            if (q.phase == 0) {
                if (mw < 0.0) {
                    q.have_lo = true;
                    q.lo = q.cur;
                    q.lo_min = mw;
                    q.phase = 1;
                    if (newton) need_d.push_back(b);
                } else {
                    q.have_hi = true;
                    q.hi = q.cur;
                    q.hi_min = mw;
                    std::vector<int> one_b(1, b);
                    BWork w1;
                    BRC(bt.make_work(one_b, one, false, w1));
                    launch_copy_b(bt.s, bt.d, w1.plist, 1, bt.maxpad, S.Best, S.W);  // w at hi
                }
            } else {
                if (mw < 0.0) {
                    q.lo = q.cur;
                    q.lo_min = mw;
                } else {
                    q.hi = q.cur;
                    q.hi_min = mw;
                    std::vector<int> one_b(1, b);
                    BWork w1;
                    BRC(bt.make_work(one_b, one, false, w1));
                    launch_copy_b(bt.s, bt.d, w1.plist, 1, bt.maxpad, S.Best, S.W);
                    if (mw < q.eps) q.phase = 2;  // halting rule: 0 <= min w < eps
                }
                if (newton && q.phase == 1) need_d.push_back(b);
            }
        }
        if (!need_d.empty()) {
            // (D o Z) w with the factor of this step, then Z^{-1} of it
            BWork wz, wr, w1;
            BRC(bt.make_work(need_d, [&](int p) { return dz_b_units(bt.h[p].n); }, false, wz));
            BRC(bt.make_work(need_d, [&](int p) { return bt.h[p].npad / 256; }, false, wr));
            BRC(bt.make_work(need_d, one, false, w1));
            for (int b = 0; b < B; ++b) bt.h[b].active = 0;
            for (int b : need_d) bt.h[b].active = 1;
            BRC(bt.upload_desc());
            launch_dzmv_b(bt.s, bt.m, bt.d, wz, wr, S.DZ, S.Rhs);
            launch_amax_b(bt.s, bt.d, w1.plist, w1.na, S.Rhs, SC_AMAX);
            std::vector<double> am;
            BRC(bt.gather(w1.plist, w1.na, SC_AMAX, 1, am));
            std::vector<double> bnd(B, 1.0);
            for (size_t i = 0; i < need_d.size(); ++i) bnd[need_d[i]] = am[i];
            std::vector<BRefine> st2;
            BRC(batch_refine(bt, need_d, S.Rhs, bnd, o, st2));
            BWork w2;
            BRC(bt.make_work(need_d, one, false, w2));
            launch_pick_b(bt.s, bt.d, w2.plist, w2.na, S.Best, SC_SUM + 2, SC_PICK);
            std::vector<double> dd;
            BRC(bt.gather(w2.plist, w2.na, SC_PICK, 1, dd));
            for (size_t i = 0; i < need_d.size(); ++i) {
                Cloud &q = cl[need_d[i]];
                q.last_d = dd[i];
                q.last_has_d = std::isfinite(dd[i]);
            }
        }
    }
    // outputs
    std::vector<int> ids;
    for (int b = 0; b < B; ++b) {
        t_plus[b] = (cl[b].no_sign || !cl[b].have_lo) ? 0.0 : cl[b].hi;
        if (w && !cl[b].no_sign && cl[b].have_lo) ids.push_back(b);
        if (info) {
            mag_tplus_info &f = info[b];
            std::memset(&f, 0, sizeof(f));
            f.t_plus = t_plus[b];
            f.t_bound = cl[b].tb;
            f.d_min = cl[b].dmin;
            f.min_w = cl[b].hi_min;
            f.t_bracket_lo = cl[b].lo;
            f.t_bracket_hi = cl[b].hi;
            f.solves = cl[b].solves;
            f.newton_steps = cl[b].newton_steps;
            f.no_sign_change = (cl[b].no_sign || !cl[b].have_lo) ? 1 : 0;
            f.status = MAG_OK;
        }
    }
    if (!ids.empty()) {
        for (int b = 0; b < B; ++b) bt.h[b].active = 1;
        BRC(bt.upload_desc());
        BWork w1;
        BRC(bt.make_work(ids, one, false, w1));
        std::vector<int64_t> po;
        for (int b : ids) po.push_back(offs[b] - offs[0]);
        const int64_t *po_dev = bt.put(po, false);
        if (!po_dev) return MAG_ENOMEM;
        launch_unpack_b(bt.s, bt.d, w1.plist, w1.na, po_dev, S.W, w, bt.maxn);
        BRC(bt.sync());
    }
    return MAG_OK;
}

}  // extern "C"
