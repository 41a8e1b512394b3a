// CG on several lattices of unequal volume at once (thermal lattices are small,
// paper section 2.1: a thermal lattice uses less parallelism).  Each stage of
// a CG iteration on Mhat^+ Mhat is a single grid-stride launch over the tiles
// of all lattices, every lattice with its own solver state; lattices that have
// converged are skipped inside the launches.  An iteration is 4 hop launches
// (the first tile of a lattice finishing the previous beta in the first and its
// alpha reduction in the third) and the search-direction update, which forms
// beta itself and leaves the state's beta finish pending; the
// iterations queued between two host checks can be captured once in a
// hipGraph and replayed with one launch, which removes the per-kernel launch
// cost of the host at these volumes.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "device.h"
#include "internal.h"
#include "ops.h"

namespace tmqcd {
namespace {

constexpr int kPersistentGrid = 1024;   // blocks of a batched launch (4 per CU)

struct Lat {
    Geom g;
    OpCtx c;
    CgState* st;
    double* partials;
    char *r, *p, *ax, *t1, *t2, *t3;
};

int64_t al(int64_t v) { return round_up(v, kAlignBytes); }

// [n solver states][per lattice: partials, r, p, ax, t1, t2, t3]
std::vector<Lat> carve(int n, const tmqcd_problem* probs, char* base, int64_t* total) {
    std::vector<Lat> L(n);
    int64_t off = al((int64_t)n * al(sizeof(CgState)));
    for (int i = 0; i < n; ++i) {
        Lat& l = L[i];
        l.g = make_geom(probs[i]);
        l.st = base ? reinterpret_cast<CgState*>(base + i * al(sizeof(CgState))) : nullptr;
        auto take = [&](int64_t bytes) {
            char* q = base ? base + off : nullptr;
            off += al(bytes);
            return q;
        };
        l.partials = reinterpret_cast<double*>(take(partial_bytes(l.g)));
        const int64_t hb = half_field_bytes(l.g, TMQCD_F64);
        l.r = take(hb);
        l.p = take(hb);
        l.ax = take(hb);
        l.t1 = take(hb);
        l.t2 = take(hb);   // t1, t2 contiguous: the operator's temporaries
        l.t3 = take(hb);
    }
    if (total) *total = off;
    return L;
}

StateInit none() {
    StateInit v;
    std::memset(&v, 0, sizeof(v));
    return v;
}

}  // namespace

int64_t cg_batch_workspace(int n, const tmqcd_problem* probs) {
    int64_t total = 0;
    carve(n, probs, nullptr, &total);
    return total;
}

#define TRY(expr)                          \
    do {                                   \
        hipError_t e_ = (expr);            \
        if (e_ != hipSuccess) {            \
            g_last_hip_error = (int)e_;    \
            rc = TMQCD_EHIP;               \
            goto done;                     \
        }                                  \
    } while (0)

int run_cg_batch(int n, const tmqcd_problem* probs, const void* const* gauge, const void* const* b, void* const* x,
                 const tmqcd_cg_opts& o, tmqcd_cg_stats* stats, bool use_graph, void* ws, hipStream_t user_stream) {
    const auto t0 = std::chrono::steady_clock::now();
    int rc = TMQCD_OK;
    hipStream_t s = user_stream;
    bool own_stream = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<Lat> L = carve(n, probs, static_cast<char*>(ws), nullptr);
    std::vector<CgState> hs(n);
    std::vector<double> bb(n, 0.0);
    std::vector<int> applies(n, 0), active(n, 1);
    std::vector<HopParams> k1(n), k2(n), k3(n), k4(n);
    std::vector<VecSpec> vs(n);
    std::vector<void*> pp(n), xp(n);
    std::vector<const void*> rp(n);
    std::vector<CgState*> sp(n);
    const int check = o.check_every > 0 ? o.check_every : 8;
    auto read_states = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int i = 0; i < n && e == hipSuccess; ++i)
            e = hipMemcpyAsync(&hs[i], L[i].st, sizeof(CgState), hipMemcpyDeviceToHost, s);
        return e == hipSuccess ? hipStreamSynchronize(s) : e;
    };
    std::vector<const double*> parts(n);
    std::vector<int> nb(n);
    auto iteration = [&]() -> hipError_t {
        for (int i = 0; i < n; ++i) {   // each lattice's first tile finishes the previous beta, if pending
            k1[i].fin_partials = parts[i];
            k1[i].fin_n = nb[i];
            k1[i].fin_kind = kFinishBetaPending;
        }
        hipError_t e = launch_hop_batch(k1.data(), n, kPersistentGrid, s);
        if (e == hipSuccess) e = launch_hop_batch(k2.data(), n, kPersistentGrid, s, nb.data());
        for (int i = 0; i < n; ++i) {   // each lattice's first tile of the next stage finishes alpha
            k3[i].fin_partials = parts[i];
            k3[i].fin_n = nb[i];
            k3[i].fin_kind = kFinishAlpha;
        }
        if (e == hipSuccess) e = launch_hop_batch(k3.data(), n, kPersistentGrid, s);
        if (e == hipSuccess) e = launch_hop_batch(k4.data(), n, kPersistentGrid, s, nb.data());
        // x += alpha p and p = r + beta p, beta formed from the update's partials; the beta finish is pending
        if (e == hipSuccess)
            e = launch_xpay_batch(vs.data(), pp.data(), rp.data(), xp.data(), sp.data(), parts.data(), nb.data(), n,
                                  kPersistentGrid, s);
        return e;
    };
    // the pending beta finish of the last iteration queued (before the host reads the states)
    auto finish_pending = [&]() -> hipError_t {
        return nb[0] > 0 ? launch_cg_finish_batch(sp.data(), parts.data(), nb.data(), n, kFinishBetaPending, s)
                         : hipSuccess;
    };
    // a stream that can be captured (the null stream cannot)
    if (use_graph && s == nullptr) {
        TRY(hipStreamCreate(&s));
        own_stream = true;
    }
    for (int i = 0; i < n; ++i) {
        Lat& l = L[i];
        l.c = make_ctx(probs[i], TMQCD_F64, o.recon, gauge[i], s);
        vs[i] = VecSpec{&l.g, 1};
        StateInit v = none();
        v.set_iter = v.set_max_iter = v.set_cycle_end = v.set_done = true;
        v.max_iter = o.max_iter;
        v.cycle_end = o.max_iter;
        v.done = kDoneRunning;
        TRY(launch_set_state(l.st, v, s));
        TRY(launch_zero(vs[i], x[i], TMQCD_F64, s));
        TRY(launch_convert(vs[i], l.r, TMQCD_F64, b[i], TMQCD_F64, s));
        TRY(launch_convert(vs[i], l.p, TMQCD_F64, b[i], TMQCD_F64, s));
        TRY(launch_norm2(vs[i], l.r, TMQCD_F64, l.st, 0, l.partials, s));
        TRY(launch_norm2(vs[i], b[i], TMQCD_F64, l.st, 1, l.partials, s));
        k1[i] = hp_schur_first(l.c, l.p, l.t1, false, kOne);
        k1[i].st = l.st;
        k2[i] = hp_schur_second(l.c, l.t1, l.p, l.t2, false, kEpiStoreNorm, l.st, l.partials, nullptr, nullptr, nullptr,
                                kOne);
        k3[i] = hp_schur_first(l.c, l.t2, l.t3, true, kOne);
        k3[i].st = l.st;
        k4[i] = hp_schur_second(l.c, l.t3, l.t2, nullptr, true, kEpiCgUpdate, l.st, l.partials, nullptr, l.r, nullptr,
                                kOne);
        parts[i] = l.partials;
        pp[i] = l.p;
        xp[i] = x[i];
        rp[i] = l.r;
        sp[i] = l.st;
    }
    TRY(read_states());
    for (int i = 0; i < n; ++i) {
        std::memset(&stats[i], 0, sizeof(tmqcd_cg_stats));
        bb[i] = hs[i].result[1];
        const double rr = hs[i].result[0];
        if (!std::isfinite(rr) || !std::isfinite(bb[i])) {
            rc = TMQCD_EBREAKDOWN;
            goto done;
        }
        StateInit v = none();
        v.set_rr = v.set_stop = v.set_done = true;
        v.rr = rr;
        v.stop_rr = o.tol * o.tol * bb[i];
        // b = 0: x = 0 is exact; the lattice is skipped from the start
        v.done = bb[i] == 0.0 ? kDoneStop : kDoneRunning;
        if (bb[i] == 0.0) {
            active[i] = 0;
            stats[i].converged = 1;
        }
        TRY(launch_set_state(L[i].st, v, s));
    }
    if (use_graph) {   // one graph holds all the iterations queued between two host checks
        TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t ec = hipSuccess;
        for (int k = 0; k < check && ec == hipSuccess; ++k) ec = iteration();
        if (ec == hipSuccess) ec = finish_pending();   // each replay ends finished
        const hipError_t ee = hipStreamEndCapture(s, &graph);
        TRY(ec);
        TRY(ee);
        TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    for (;;) {
        bool any = false;
        for (int i = 0; i < n; ++i) any = any || active[i];
        if (!any) break;
        // iterate until every active lattice has stopped
        for (;;) {
            if (use_graph) {
                TRY(hipGraphLaunch(exec, s));
            } else {
                for (int k = 0; k < check; ++k) TRY(iteration());
                TRY(finish_pending());
            }
            TRY(read_states());
            bool running = false;
            for (int i = 0; i < n; ++i) running = running || (active[i] && hs[i].done == kDoneRunning);
            if (!running) break;
        }
        // FP64 residual of every lattice that stopped; restart those above tolerance
        for (int i = 0; i < n; ++i) {
            if (!active[i]) continue;
            Lat& l = L[i];
            TRY(apply_operator(l.c, TMQCD_MHATDAGMHAT, x[i], l.ax, l.t1, 1));
            ++applies[i];
            TRY(launch_residual(vs[i], l.r, b[i], l.ax, l.st, 0, l.partials, s));
        }
        TRY(read_states());
        for (int i = 0; i < n; ++i) {
            if (!active[i]) continue;
            const double rr_true = hs[i].result[0];
            stats[i].iters = hs[i].iter;
            stats[i].reliable_updates += 1;
            stats[i].iter_rel_residual = std::sqrt(hs[i].rr / bb[i]);
            stats[i].true_rel_residual = std::sqrt(rr_true / bb[i]);
            if (rr_true <= o.tol * o.tol * bb[i]) {
                stats[i].converged = 1;
                active[i] = 0;
                continue;
            }
            if (!std::isfinite(rr_true) || hs[i].done == kDoneBreakdown) {
                rc = TMQCD_EBREAKDOWN;
                active[i] = 0;
                continue;
            }
            if (hs[i].iter >= o.max_iter) {
                if (rc == TMQCD_OK) rc = TMQCD_ENOCONV;
                active[i] = 0;
                continue;
            }
            // restart from the true residual, keeping the search direction
            StateInit v = none();
            v.set_beta = v.set_done = v.set_rr = true;
            v.beta = rr_true / (hs[i].rr_prev > 0 ? hs[i].rr_prev : rr_true);
            v.rr = rr_true;
            v.done = kDoneRunning;
            TRY(launch_set_state(L[i].st, v, s));
            TRY(launch_xpay(vs[i], L[i].p, TMQCD_F64, L[i].r, TMQCD_F64, L[i].st, false, s));
        }
        // stopped lattices keep done != 0, so the batched launches skip them
        for (int i = 0; i < n; ++i)
            if (!active[i]) {
                StateInit v = none();
                v.set_done = true;
                v.done = kDoneStop;
                TRY(launch_set_state(L[i].st, v, s));
            }
    }
    for (int i = 0; i < n; ++i) stats[i].hop_launches = 4 * (stats[i].iters + applies[i]);
    TRY(hipStreamSynchronize(s));
done:   // teardown: the status is already decided, so errors here are dropped
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (own_stream) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < n; ++i) stats[i].seconds = secs;
    return rc;
}

#undef TRY

}  // namespace tmqcd
