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

    // Append bytes to an arena region.  Transient data: the host copy is made
    // now and the device copy enqueued on the stream (pinned source); they are
    // reset at every host sync (all copies done by then).  Persistent data (the
    // step graph's work lists and states): only the host copy is made; one
    // flush_persistent() uploads the whole region before anything reads it.
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
            if (!persist && hipMemcpyAsync(dp, hp, v.size() * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess)
                return nullptr;
        }
        used += bytes;
        return reinterpret_cast<T *>(dp);
    }
    int flush_persistent()
    {
        if (persist_used == 0) return MAG_OK;
        return hipMemcpyAsync(dev_arena, host_arena, persist_used, hipMemcpyHostToDevice, s) == hipSuccess
                   ? MAG_OK
                   : MAG_EHIP;
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

// split-reduction doubles of one problem: products, derivatives, dot products, d_min
size_t batch_partial_doubles(int64_t n, int restart)
{
    size_t p = std::max(zmv_partial_doubles(n), pair_partial_doubles(n, 1));
    p = std::max(p, blas1_partial_doubles(restart + 2));
    p = std::max(p, dmin_partial_doubles(n) + 8);
    return p + 64;
}

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
        part += batch_partial_doubles(ns[b], restart);
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
        pp += batch_partial_doubles(ns[b], restart);
        q.ints = (int *)c->bints.p + (size_t)b * kIntsPer;
        q.m = m;
        q.active = 1;
    }
    BCHK(hipMemsetAsync(c->bvec.p, 0, sizeof(double) * vec, bt.s));
    BCHK(hipMemsetAsync(c->bscal.p, 0, sizeof(double) * (size_t)B * SC_COUNT, bt.s));
    BCHK(hipMemsetAsync(c->bints.p, 0, sizeof(int) * (size_t)B * kIntsPer, bt.s));
    return bt.upload_desc();
}

// The factorisation schedule of all problems (work lists in the persistent
// arena), launched inside the step graph's capture; every kernel skips problems
// whose descriptor is inactive.
struct FLaunch {
    int kind;  // 0 trsm, 1 subupdate, 2 syrk (pair), 3 potrf, 4 tilegen, 5 zero status, 6 strip, 7 syrk (single)
    int64_t kk;
    BWork w;
};

// group: 0 the context's tuned choice for this batch's largest npad, 1 single
// panels, 2 pairs.
int batch_factor_schedule(Batch &bt, std::vector<FLaunch> &seq, int group = 0)
{
    std::vector<int> all(bt.B);
    for (int b = 0; b < bt.B; ++b) all[b] = b;
    BWork wall;
    BRC(bt.make_work(all, [&](int) { return (int64_t)1; }, true, wall));
    seq.push_back({5, 0, wall});
    BWork wt;
    BRC(bt.make_work(all, [&](int p) { return tilegen32_blocks(bt.h[p].npad); }, true, wt));
    seq.push_back({4, 0, wt});
    if (group == 0) group = bt.c->tune_bgroup[size_bucket(bt.maxpad)];
    if (group == 1) {
        // single panels of kPanel columns: two 128-column sub-panels, then one
        // trailing update with K = 256
        for (int64_t k = 0; k < bt.maxpad; k += kPanel) {
            for (int sub = 0; sub < kPanel / kTile; ++sub) {
                const int64_t kk = k + sub * kTile;
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
            BWork w4;
            BRC(bt.make_work(all, [&](int p) { return k < bt.h[p].npad ? gemm_b_units(4, bt.h[p].npad, k) : 0; }, true, w4));
            seq.push_back({7, k, w4});
        }
        return MAG_OK;
    }
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
    return MAG_OK;
}

void record_factor(Batch &bt, const std::vector<FLaunch> &seq)
{
    for (const FLaunch &L : seq) {
        switch (L.kind) {
        case 5: launch_zero_status_b(bt.s, bt.d, L.w.plist, L.w.na); break;
        case 4: launch_tilegen32_b(bt.s, bt.d, L.w); break;
        case 3: launch_potrf128_b(bt.s, bt.d, L.w, L.kk); break;
        case 6: launch_gemm_b(bt.s, 3, bt.d, L.w, L.kk); break;
        case 7: launch_gemm_b(bt.s, 4, bt.d, L.w, L.kk); break;
        default: launch_gemm_b(bt.s, L.kind, bt.d, L.w, L.kk); break;
        }
    }
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

// Work lists of the step graph's products over all problems (persistent arena).
struct AllWork {
    const int *all = nullptr;  // 0..B-1
    BWork wz, wr, wp, wdz, wdr;
};

int make_all_work(Batch &bt, AllWork &A)
{
    std::vector<int> all(bt.B);
    for (int b = 0; b < bt.B; ++b) all[b] = b;
    BRC(bt.make_work(all, [&](int p) { return zmv_b_units(bt.h[p].n, bt.m); }, true, A.wz));
    BRC(bt.make_work(all, [&](int p) { return zmv_b_reduce_units(bt.h[p].n, bt.m); }, true, A.wr));
    BRC(bt.make_work(all, [&](int p) { return prec_b_units(bt.h[p].npad); }, true, A.wp));
    BRC(bt.make_work(all, [&](int p) { return dz_b_units(bt.h[p].n); }, true, A.wdz));
    BRC(bt.make_work(all, [&](int p) { return bt.h[p].npad / 256; }, true, A.wdr));
    A.all = bt.put(all, true);
    return A.all ? MAG_OK : MAG_ENOMEM;
}

struct RefPlan {
    int rounds = 4;      // correction rounds (each a residual, then a plain step or a GMRES cycle)
    int kcycle = 12;     // Arnoldi steps per GMRES cycle
    int max_gmres = 200;
    double tol = 1e-12, inner_tol = 1e-10;
};

// Record the device-controlled refinement of Z x = b (b in rhs_slot, zero
// padded) for the problems active on entry; the best iterate lands in slot
// Best.  bnorm_off: scalar slot of ||b||_inf (tol scales with it), or -1.
void record_refine(Batch &bt, const AllWork &A, int rhs_slot, int64_t bnorm_off, const RefPlan &rp)
{
    const Slots &S = bt.sl;
    hipStream_t s = bt.s;
    BProb *P = bt.d;
    const int B = bt.B;
    const int64_t mp = bt.maxpad;
    launch_ref_init_b(s, P, B, bnorm_off, rp.tol);
    launch_gate_b(s, P, B, F_REF);
    launch_prec_apply_b(s, P, A.wp, rhs_slot, S.Y, S.X);  // x0 = M^{-1} b
    for (int round = 0; round <= rp.rounds; ++round) {
        const int final_round = round == rp.rounds ? 1 : 0;
        launch_gate_b(s, P, B, F_REF);
        launch_zmv_b(s, bt.m, P, A.wz, A.wr, S.X, S.Rr, rhs_slot, 1, SC_RNORM);
        launch_ref_decide_b(s, P, B, final_round, rp.max_gmres);
        launch_gate_b(s, P, B, F_COPYBEST);
        launch_copy_b(s, P, A.all, B, mp, S.X, S.Best);
        if (final_round) break;
        if (round > 0) {  // the first round cannot revert (no best iterate before it)
            launch_gate_b(s, P, B, F_REVERT);
            launch_copy_b(s, P, A.all, B, mp, S.Best, S.X);
        }
        launch_gate_b(s, P, B, F_DOPLAIN);
        launch_prec_apply_b(s, P, A.wp, S.Rr, S.Y, S.Z);
        launch_axpy_slot_b(s, P, B, mp, S.Z, S.X);
        // the first round's correction is always a plain step (plain mode starts
        // on, and a switch to GMRES needs a plain step that gained too little)
        if (round == 0) continue;
        launch_gate_b(s, P, B, F_DOGMRES);
        launch_prec_apply_b(s, P, A.wp, S.Rr, S.Y, S.Z);
        launch_nrm2_b(s, P, A.all, B, S.Z, SC_BETA);
        launch_gmres_start_b(s, P, B);
        launch_gate_b(s, P, B, F_INNER);
        launch_scale_inv_b(s, P, A.all, B, mp, S.Z, S.V0, SC_BETA);
        for (int k = 0; k < rp.kcycle; ++k) {
            launch_gate_b(s, P, B, F_INNER);
            launch_zmv_b(s, bt.m, P, A.wz, A.wr, S.V0 + k, S.U, -1, 0, 0);
            launch_prec_apply_b(s, P, A.wp, S.U, S.Y, S.V0 + k + 1);
            launch_arnoldi_b(s, P, B, k, S.V0, rp.kcycle, rp.inner_tol, rp.max_gmres);
        }
        launch_gmres_finish_b(s, P, B, rp.kcycle);
        launch_gate_b(s, P, B, F_DOGMRES);
        launch_multi_axpy_b(s, P, A.all, B, mp, S.V0, rp.kcycle, SC_Y, S.X, 1.0);
    }
}

// Capture one step of the batched search (or of the fixed-scale solves) as a
// graph: each cloud's next scale, the factorisation, the refinement, min w,
// the bracket update and, for Newton steps, d(min w)/dt; then the count of
// clouds still searching into dcount[0..2).
int build_step_graph(Batch &bt, const std::vector<FLaunch> &fseq, const AllWork &A, SState *S, const SParams &prm,
                     const RefPlan &rp, const RefPlan &dp, int *dcount)
{
    const Slots &SL = bt.sl;
    hipStream_t s = bt.s;
    BProb *P = bt.d;
    const int B = bt.B;
    const int64_t mp = bt.maxpad;
    BRC(bt.flush_persistent());     // work lists and states, in one copy
    BCHK(hipStreamSynchronize(s));
    BCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    launch_search_select_b(s, P, S, B, prm);
    record_factor(bt, fseq);
    launch_breakdown_b(s, P, S, B);
    launch_gate_b(s, P, B, F_SEARCH);
    launch_fill_b(s, P, A.all, B, mp, SL.Rhs, 1.0, true);
    record_refine(bt, A, SL.Rhs, -1, rp);
    launch_gate_b(s, P, B, F_SEARCH);
    launch_summin_b(s, P, A.all, B, SL.Best, SC_SUM);
    launch_search_update_b(s, P, S, B, prm);
    launch_gate_b(s, P, B, F_HI);
    launch_copy_b(s, P, A.all, B, mp, SL.Best, SL.W);
    if (prm.newton) {
        // dw/dt = Z^{-1} (D o Z) w with this step's factor; its entry at argmin w
        launch_gate_b(s, P, B, F_NEEDD);
        launch_copy_b(s, P, A.all, B, mp, SL.Best, SL.DZ);
        launch_dzmv_b(s, bt.m, P, A.wdz, A.wdr, SL.DZ, SL.Rhs);
        launch_amax_b(s, P, A.all, B, SL.Rhs, SC_AMAX);
        record_refine(bt, A, SL.Rhs, SC_AMAX, dp);
        launch_gate_b(s, P, B, F_NEEDD);
        launch_pick_b(s, P, A.all, B, SL.Best, SC_SUM + 2, SC_PICK);
        launch_search_deriv_b(s, P, S, B);
    }
    launch_search_count_b(s, S, B, dcount);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(s, &g) != hipSuccess) return MAG_EHIP;
    bt.graph_def = g;
    BCHK(hipGraphInstantiate(&bt.graph, g, nullptr, nullptr, 0));
    return MAG_OK;
}

// Run step graphs until no cloud is searching (one count read per step).
// Returns the number of steps, or a negative error code.
int run_steps(Batch &bt, const int *dcount, int max_steps)
{
    int *hc = reinterpret_cast<int *>(bt.c->host_scalars + 60);
    for (int step = 0; step < max_steps; ++step) {
        BCHK(hipGraphLaunch(bt.graph, bt.s));
        BCHK(hipMemcpyAsync(hc, dcount, 2 * sizeof(int), hipMemcpyDeviceToHost, bt.s));
        BCHK(hipStreamSynchronize(bt.s));
        if (hc[1]) return MAG_ENOTPD;  // the FP32 factor broke down at every shift
        if (hc[0] == 0) return step + 1;
    }
    return MAG_ENOCONV;
}

// Checks of every cloud in one pass: finite coordinates (MAG_EINVAL) and the
// squared minimum distance by brute force (0: coincident points, MAG_ENOTPD),
// returned in dmin2.  One host sync.
int batch_validate(Batch &bt, std::vector<double> &dmin2)
{
    mag_ctx *c = bt.c;
    int *status = (int *)c->ints.p;
    launch_fill_ints(bt.s, status, 8, 0);
    std::vector<int> pl;
    for (int b = 0; b < bt.B; ++b) {
        const BProb &q = bt.h[b];
        launch_check_finite(bt.s, q.X, q.n * (int64_t)bt.m, status);
        if (q.n >= 2) {
            launch_dmin2(bt.s, q.X, q.n, bt.m, q.partial, nullptr, q.scal + SC_PICK);
            pl.push_back(b);
        }
    }
    BCHK(hipMemcpyAsync(c->host_scalars + 56, status, 8 * sizeof(int), hipMemcpyDeviceToHost, bt.s));
    dmin2.assign(bt.B, INFINITY);
    if (!pl.empty()) {
        const int *pd = bt.put(pl, false);
        if (!pd) return MAG_ENOMEM;
        std::vector<double> v;
        BRC(bt.gather(pd, (int)pl.size(), SC_PICK, 1, v));
        for (size_t i = 0; i < pl.size(); ++i) dmin2[pl[i]] = v[i];
    } else {
        BRC(bt.sync());
    }
    if (((const int *)(c->host_scalars + 56))[kStNonFinite]) return MAG_EINVAL;
    for (int b = 0; b < bt.B; ++b)
        if (!(dmin2[b] > 0.0)) return MAG_ENOTPD;
    return MAG_OK;
}

RefPlan main_plan(const mag_opts &o, int restart)
{
    RefPlan rp;
    rp.rounds = std::max(1, std::min(o.max_outer, 4));  // one plain round, then three that may run GMRES
    rp.kcycle = std::max(1, std::min(restart, 12));
    rp.max_gmres = o.max_gmres > 0 ? o.max_gmres : 200;
    rp.tol = o.tol > 0 ? o.tol : 1e-12;
    rp.inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-10;
    return rp;
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
        if (ns[b] < 1) return MAG_EINVAL;
    }
    Batch bt;
    const int restart = std::min(kMaxRestart, std::max(1, o.gmres_restart));
    BRC(batch_setup(c, bt, Xs, ns, m, ts, restart));
    std::vector<double> dmin2;
    BRC(batch_validate(bt, dmin2));
    // one fixed-scale solve per problem, retried with a shift after an FP32 breakdown
    std::vector<SState> st0(B);
    std::memset(st0.data(), 0, sizeof(SState) * B);
    SState *Sd = bt.put(st0, true);
    if (!Sd) return MAG_ENOMEM;
    std::vector<FLaunch> fseq;
    BRC(batch_factor_schedule(bt, fseq));
    AllWork A;
    BRC(make_all_work(bt, A));
    SParams prm{};
    prm.fixed = 1;
    int *dcount = reinterpret_cast<int *>(bt.dstage + (size_t)B * 128);
    const RefPlan rp = main_plan(o, restart);
    BRC(build_step_graph(bt, fseq, A, Sd, prm, rp, rp, dcount));
    const int steps = run_steps(bt, dcount, 8);
    if (steps < 0) return steps;
    std::vector<SState> st(B);
    BCHK(hipMemcpyAsync(st.data(), Sd, sizeof(SState) * B, hipMemcpyDeviceToHost, bt.s));
    std::vector<int> all(B);
    for (int b = 0; b < B; ++b) all[b] = b;
    BWork w1;
    BRC(bt.make_work(all, [](int) { return (int64_t)1; }, false, w1));
    std::vector<double> rc;
    BRC(bt.gather(w1.plist, w1.na, SC_RC, 8, rc));
    // items the graph's rounds did not take to tol: the host-driven refinement
    // from scratch with the factor in place (GMRES with the caller's limits)
    std::vector<int> redo;
    for (int b = 0; b < B; ++b)
        if (st[b].unconverged) redo.push_back(b);
    std::vector<BRefine> fb;
    if (!redo.empty()) {
        for (int b = 0; b < B; ++b) bt.h[b].active = 0;
        for (int b : redo) bt.h[b].active = 1;
        BRC(bt.upload_desc());
        BWork wr;
        BRC(bt.make_work(redo, [](int) { return (int64_t)1; }, false, wr));
        launch_fill_b(bt.s, bt.d, wr.plist, wr.na, bt.maxpad, bt.sl.Rhs, 1.0, true);
        std::vector<double> bn(B, 1.0);
        BRC(batch_refine(bt, redo, bt.sl.Rhs, bn, o, fb));
    }
    for (int b = 0; b < B; ++b) bt.h[b].active = 1;
    BRC(bt.upload_desc());
    // transient lists do not outlive a sync (the gathers above reset the arena)
    BWork wo;
    BRC(bt.make_work(all, [](int) { return (int64_t)1; }, false, wo));
    std::vector<int64_t> po(B);
    for (int b = 0; b < B; ++b) po[b] = offs[b] - offs[0];
    const int64_t *po_dev = bt.put(po, false);
    if (!po_dev) return MAG_ENOMEM;
    launch_unpack_b(bt.s, bt.d, wo.plist, wo.na, po_dev, bt.sl.Best, w, bt.maxn);
    launch_summin_b(bt.s, bt.d, wo.plist, wo.na, bt.sl.Best, SC_SUM);
    std::vector<double> sums;
    BRC(bt.gather(wo.plist, wo.na, SC_SUM, 3, sums));
    int rc_all = MAG_OK;
    for (int b = 0; b < B; ++b) {
        const bool redone = st[b].unconverged != 0;
        const bool ok = redone ? fb[b].ok != 0 : true;
        if (M) M[b] = sums[3 * b];
        if (!ok) rc_all = MAG_ENOCONV;
        if (info) {
            mag_info &f = info[b];
            std::memset(&f, 0, sizeof(f));
            f.status = ok ? MAG_OK : MAG_ENOCONV;
            f.outer_iters = redone ? fb[b].outer : (int)rc[8 * b + RC_ROUND];
            f.gmres_iters = redone ? fb[b].inner : (int)rc[8 * b + RC_INNER];
            f.shifted = st[b].shift > 0.0 ? 1 : 0;
            f.shift = st[b].shift;
            f.resid_inf = redone ? fb[b].best : rc[8 * b + RC_BEST];
            f.magnitude = sums[3 * b];
            f.min_w = sums[3 * b + 1];
            f.argmin_w = (int64_t)sums[3 * b + 2];
            f.solver = MAG_FP32_IR;
        }
    }
    return rc_all;
}

// ---- tuning of the batched factorisation ---------------------------------------

int mag_tune_batch_group(mag_ctx *c, int64_t max_n, int32_t group)
{
    if (!c || max_n < 1 || group < 0 || group > 2) return MAG_EINVAL;
    c->tune_bgroup[size_bucket(round_up(max_n, kPad))] = group;
    return MAG_OK;
}

int mag_autotune_batch(mag_ctx *c, int32_t B, const double *X, const int64_t *offs, int32_t m, const double *t,
                       int32_t reps, int32_t *group_out, double *ms_out)
{
    if (!c || B < 1 || !X || !offs || !t || m < 1) return MAG_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return MAG_EHIP;
    std::vector<const double *> Xs(B);
    std::vector<int64_t> ns(B);
    std::vector<double> ts(B);
    for (int b = 0; b < B; ++b) {
        if (offs[b + 1] <= offs[b] || !(std::isfinite(t[b]) && t[b] > 0.0)) return MAG_EINVAL;
        Xs[b] = X + offs[b] * m;
        ns[b] = offs[b + 1] - offs[b];
        ts[b] = t[b];
    }
    Batch bt;
    BRC(batch_setup(c, bt, Xs, ns, m, ts, 1));
    std::vector<double> dmin2;
    BRC(batch_validate(bt, dmin2));
    // the two schedules' launch sequences, each captured into a graph of its own
    hipGraph_t gdef[2] = {nullptr, nullptr};
    hipGraphExec_t gexe[2] = {nullptr, nullptr};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best[2] = {INFINITY, INFINITY};
    int rc = MAG_OK;
    std::vector<FLaunch> seq[2];
    for (int q = 0; q < 2 && rc == MAG_OK; ++q) rc = batch_factor_schedule(bt, seq[q], q + 1);
    if (rc == MAG_OK) rc = bt.flush_persistent();
    if (rc == MAG_OK && hipStreamSynchronize(bt.s) != hipSuccess) rc = MAG_EHIP;
    for (int q = 0; q < 2 && rc == MAG_OK; ++q) {
        if (hipStreamBeginCapture(bt.s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = MAG_EHIP;
            break;
        }
        record_factor(bt, seq[q]);
        if (hipStreamEndCapture(bt.s, &gdef[q]) != hipSuccess ||
            hipGraphInstantiate(&gexe[q], gdef[q], nullptr, nullptr, 0) != hipSuccess)
            rc = MAG_EHIP;
    }
    if (rc == MAG_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = MAG_EHIP;
    for (int rep = 0; rep < std::max(1, reps) && rc == MAG_OK; ++rep) {
        for (int q = 0; q < 2; ++q) {
            float ms = 0.0f;
            if (hipEventRecord(e0, bt.s) != hipSuccess || hipGraphLaunch(gexe[q], bt.s) != hipSuccess ||
                hipEventRecord(e1, bt.s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = MAG_EHIP;
                break;
            }
            best[q] = std::min(best[q], (double)ms);
        }
    }
    for (int q = 0; q < 2; ++q) {
        if (gexe[q]) hipGraphExecDestroy(gexe[q]);
        if (gdef[q]) hipGraphDestroy(gdef[q]);
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (rc != MAG_OK) return rc;
    const int pick = best[0] < best[1] ? 1 : 2;
    c->tune_bgroup[size_bucket(bt.maxpad)] = pick;
    if (group_out) *group_out = pick;
    if (ms_out) {
        ms_out[0] = best[0];
        ms_out[1] = best[1];
    }
    return MAG_OK;
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
        if (ns[b] < 1) return MAG_EINVAL;
    }
    const bool ridders = to.method == MAG_TPLUS_RIDDERS;
    Batch bt;
    const int restart = std::min(kMaxRestart, std::max(1, o.gmres_restart));
    BRC(batch_setup(c, bt, Xs, ns, m, std::vector<double>(B, 1.0), restart));
    std::vector<double> dmin2;
    BRC(batch_validate(bt, dmin2));
    // each cloud's search state: the bound t_b = log(n - 1)/d_min, the grid from it
    std::vector<SState> st0(B);
    std::memset(st0.data(), 0, sizeof(SState) * B);
    for (int b = 0; b < B; ++b) {
        SState &q = st0[b];
        if (ns[b] <= 2) {
            q.phase = 2;
            q.no_sign = 1;
            continue;
        }
        const double dm = std::sqrt(dmin2[b]);
        q.tb = std::log((double)(ns[b] - 1)) / dm;
        q.eps = to.eps > 0.0 ? to.eps : (double)ns[b] * std::ldexp(1.0, -53);
        q.top = q.tb;
        q.gi = to.grid - 1;
        q.prev_step = INFINITY;
    }
    SState *Sd = bt.put(st0, true);
    if (!Sd) return MAG_ENOMEM;
    std::vector<FLaunch> fseq;
    BRC(batch_factor_schedule(bt, fseq));
    AllWork A;
    BRC(make_all_work(bt, A));
    SParams prm{};
    prm.grid = to.grid;
    prm.max_extend = to.max_extend;
    prm.newton = (to.newton && !ridders) ? 1 : 0;
    prm.ridders = ridders ? 1 : 0;
    prm.fixed = 0;
    prm.lo_factor = to.lo_factor;
    prm.rtol = to.rtol;
    int *dcount = reinterpret_cast<int *>(bt.dstage + (size_t)B * 128);
    const RefPlan rp = main_plan(o, restart);
    RefPlan dp = rp;  // the Newton derivative: a shorter refinement suffices for a safeguarded step
    dp.rounds = std::min(rp.rounds, 2);
    dp.kcycle = std::min(rp.kcycle, 8);
    BRC(build_step_graph(bt, fseq, A, Sd, prm, rp, dp, dcount));
    const int steps = run_steps(bt, dcount, 1000);
    if (steps < 0) return steps;
    std::vector<SState> st(B);
    BCHK(hipMemcpyAsync(st.data(), Sd, sizeof(SState) * B, hipMemcpyDeviceToHost, bt.s));
    BRC(bt.sync());
    std::vector<int> ids;
    for (int b = 0; b < B; ++b) {
        const bool none = st[b].no_sign || !st[b].have_lo;
        t_plus[b] = none ? 0.0 : st[b].hi;
        if (w && !none) ids.push_back(b);
        if (info) {
            mag_tplus_info &f = info[b];
            std::memset(&f, 0, sizeof(f));
            f.t_plus = t_plus[b];
            f.t_bound = st[b].tb;
            f.d_min = std::sqrt(dmin2[b]);
            f.min_w = st[b].hi_min;
            f.t_bracket_lo = st[b].lo;
            f.t_bracket_hi = st[b].hi;
            f.solves = st[b].solves;
            f.newton_steps = st[b].newton_steps;
            f.no_sign_change = none ? 1 : 0;
            f.status = MAG_OK;
        }
    }
    if (!ids.empty()) {
        BWork w1;
        BRC(bt.make_work(ids, [](int) { return (int64_t)1; }, false, w1));
        std::vector<int64_t> po;
        for (int b : ids) po.push_back(offs[b] - offs[0]);
        const int64_t *po_dev = bt.put(po, false);
        if (!po_dev) return MAG_ENOMEM;
        launch_unpack_b(bt.s, bt.d, w1.plist, w1.na, po_dev, bt.sl.W, w, bt.maxn);
        BRC(bt.sync());
    }
    return MAG_OK;
}

}  // extern "C"
