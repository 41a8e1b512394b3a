// CG on several right-hand sides at once (the paper's section 2.1: correlators
// need one inversion per source, twelve for the spin-colour point sources of a
// propagator).  The columns share every operator application: each stage of an
// iteration is one multi-RHS hop launch that reads each link once for all
// columns, while every column keeps its own FP64 solver scalars, its own
// reductions and its own stop flag (a column that has converged is skipped by
// every launch).  FP64 throughout.
//
// One iteration on Mhat^+ Mhat (columns c = 0 .. n-1 in every launch):
//   t1_c = A^{-1} H_oe p_c
//   t2_c = A p_c - kappa^2 H_eo t1_c            and per-column |t2_c|^2 = p_c^+ Mhat^+Mhat p_c
//   finish: alpha_c = rr_c / |t2_c|^2            (one block per column)
//   t1_c = A(-mu)^{-1} H^+_oe t2_c
//   x_c += alpha_c p_c, r_c -= alpha_c (A(-mu) t2_c - kappa^2 H^+_eo t1_c), per-column |r_c|^2
//   finish: beta_c, stop tests
//   p_c = r_c + beta_c p_c
// On M^+M: t1_c = M p_c with |t1_c|^2, finish, the update after M^+, finish, p.
// The true residual b_c - A x_c is recomputed in FP64 when every running
// column has stopped; columns above tolerance restart from it (keeping their
// search direction), the others are done.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "device.h"
#include "internal.h"
#include "ops.h"

namespace tmqcd {

namespace {

int64_t al(int64_t v) { return round_up(v, kAlignBytes); }

StateInit none() {
    StateInit v;
    std::memset(&v, 0, sizeof(v));
    return v;
}

}  // namespace

// [n states][n x tiles partials of the multi-RHS launches][n x per-column partials of the set-up
// reductions][r][p][ax][t1][t2], each vector block holding the n columns one after the other
MrhsWorkspace carve_cg_mrhs(const Geom& g, int op, int n, char* base) {
    MrhsWorkspace w;
    std::memset(&w, 0, sizeof(w));
    const bool full = op == TMQCD_MDAGM;
    const int64_t hb = half_field_bytes(g, TMQCD_F64);
    w.fstride = (full ? 2 : 1) * hb;
    w.tiles_max = mrhs_tiles_max(g, full ? 2 : 1);
    w.col_partials = partial_bytes(g) / 8;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        char* p = base ? base + off : nullptr;
        off += al(bytes);
        return p;
    };
    w.st = reinterpret_cast<CgState*>(take(n * (int64_t)sizeof(CgState)));   // CgState[n], as the kernels index it
    w.partials = reinterpret_cast<double*>(take(8 * (int64_t)n * w.tiles_max));
    w.setup_partials = reinterpret_cast<double*>(take(8 * (int64_t)n * w.col_partials));
    w.r = take(n * w.fstride);
    w.p = take(n * w.fstride);
    w.ax = take(n * w.fstride);
    // the operator's temporaries: M^+M one full field per column; Mhat^+Mhat the odd t1 and the even t2
    // columns, t1 block then t2 block (the layout apply_operator expects of its nrhs temporaries)
    w.t1 = take(n * (full ? 2 * hb : hb));
    w.t2 = full ? nullptr : take(n * hb);
    w.total = off;
    return w;
}

#define TRY(expr)                                     \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) {                       \
            g_last_hip_error = (int)e_;               \
            return TMQCD_EHIP;                        \
        }                                             \
    } while (0)

int run_cg_mrhs(const tmqcd_problem& prob, const void* gauge, const void* b, void* x, const tmqcd_cg_opts& o,
                tmqcd_cg_stats* stats, void* ws, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int n = o.nrhs;
    const bool full = o.op == TMQCD_MDAGM;
    const Geom g = make_geom(prob);
    MrhsWorkspace w = carve_cg_mrhs(g, o.op, n, static_cast<char*>(ws));
    const OpCtx c = make_ctx(prob, TMQCD_F64, o.recon, gauge, s);
    const VecSpec vs{&g, full ? 2 : 1};
    const int64_t fs = w.fstride, hb = half_field_bytes(g, TMQCD_F64);
    char* xb = static_cast<char*>(x);
    const char* bb_ptr = static_cast<const char*>(b);
    const int check = o.check_every > 0 ? o.check_every : 16;
    for (int k = 0; k < n; ++k) std::memset(&stats[k], 0, sizeof(tmqcd_cg_stats));

    CgState* states = w.st;

    // set-up per column: state, x0, r = b - A x0, |b|^2, |r|^2, p = r
    for (int k = 0; k < n; ++k) {
        StateInit v = none();
        v.set_iter = v.set_max_iter = v.set_done = v.set_cycle_end = true;
        v.max_iter = o.max_iter;
        v.cycle_end = o.max_iter;
        v.done = kDoneRunning;
        TRY(launch_set_state(states + k, v, s));
    }
    int applies = 0;
    auto true_residuals = [&]() -> hipError_t {
        hipError_t e = apply_operator(c, o.op, x, w.ax, w.t1, n);
        ++applies;
        for (int k = 0; k < n && e == hipSuccess; ++k)
            e = launch_residual(vs, w.r + k * fs, bb_ptr + k * fs, w.ax + k * fs, states + k, 0,
                                w.setup_partials + k * w.col_partials, s);
        return e;
    };
    if (o.x_is_zero) {
        for (int k = 0; k < n; ++k) {
            TRY(launch_zero(vs, xb + k * fs, TMQCD_F64, s));
            TRY(launch_convert(vs, w.r + k * fs, TMQCD_F64, bb_ptr + k * fs, TMQCD_F64, s));
            TRY(launch_norm2(vs, w.r + k * fs, TMQCD_F64, states + k, 0, w.setup_partials + k * w.col_partials, s));
        }
    } else {
        TRY(true_residuals());
    }
    for (int k = 0; k < n; ++k) {
        TRY(launch_norm2(vs, bb_ptr + k * fs, TMQCD_F64, states + k, 1, w.setup_partials + k * w.col_partials, s));
        TRY(launch_convert(vs, w.p + k * fs, TMQCD_F64, w.r + k * fs, TMQCD_F64, s));
    }
    std::vector<CgState> hs(n);
    auto read_states = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(hs.data(), states, n * sizeof(CgState), hipMemcpyDeviceToHost, s);
        return e == hipSuccess ? hipStreamSynchronize(s) : e;
    };
    TRY(read_states());
    std::vector<double> bnorm(n);
    std::vector<int> active(n, 1);
    int status = TMQCD_OK;
    for (int k = 0; k < n; ++k) {
        bnorm[k] = hs[k].result[1];
        const double rr = hs[k].result[0];
        StateInit v = none();
        v.set_rr = v.set_stop = v.set_done = true;
        v.rr = rr;
        v.stop_rr = o.tol * o.tol * bnorm[k];
        v.done = kDoneRunning;
        if (!std::isfinite(rr) || !std::isfinite(bnorm[k])) {
            status = TMQCD_EBREAKDOWN;
            active[k] = 0;
            v.done = kDoneBreakdown;
        } else if (bnorm[k] == 0.0) {   // b = 0: x = 0 is exact
            TRY(launch_zero(vs, xb + k * fs, TMQCD_F64, s));
            stats[k].converged = 1;
            active[k] = 0;
            v.done = kDoneStop;
        } else if (rr <= o.tol * o.tol * bnorm[k]) {   // the start vector already solves it (true residual)
            stats[k].converged = 1;
            stats[k].true_rel_residual = stats[k].iter_rel_residual = std::sqrt(rr / bnorm[k]);
            active[k] = 0;
            v.done = kDoneStop;
        }
        TRY(launch_set_state(states + k, v, s));
    }

    // the stages of one iteration
    const Rhs one_half{n, hb, 0, hb};
    HopParams k1, k2, k3, k4;
    if (full) {
        k1 = hp_full(c, w.p, w.t1, false, kEpiStoreNorm, states, w.partials, nullptr, nullptr, nullptr,
                     Rhs{n, fs, fs, 2 * hb});
        k2 = hp_full(c, w.t1, nullptr, true, kEpiCgUpdate, states, w.partials, nullptr, w.r, nullptr,
                     Rhs{n, 2 * hb, 2 * hb, 0});
        k2.v_fstride = fs;
    } else {
        k1 = hp_schur_first(c, w.p, w.t1, false, one_half);
        k1.st = states;
        k2 = hp_schur_second(c, w.t1, w.p, w.t2, false, kEpiStoreNorm, states, w.partials, nullptr, nullptr, nullptr,
                             Rhs{n, hb, fs, hb});
        k3 = hp_schur_first(c, w.t2, w.t1, true, one_half);
        k3.st = states;
        k4 = hp_schur_second(c, w.t1, w.t2, nullptr, true, kEpiCgUpdate, states, w.partials, nullptr, w.r, nullptr,
                             Rhs{n, hb, hb, 0});
        k4.v_fstride = fs;
    }
    int hop_launches = 0;
    auto iteration = [&]() -> hipError_t {
        int tiles = 0;
        hipError_t e;
        if (full) {
            e = launch_hop(k1, s, &tiles);
            if (e == hipSuccess) e = launch_cg_finish_cols(states, w.partials, tiles, n, kFinishAlpha, s);
            if (e == hipSuccess) e = launch_hop(k2, s, &tiles);
            hop_launches += 2;
        } else {
            e = launch_hop(k1, s);
            if (e == hipSuccess) e = launch_hop(k2, s, &tiles);
            if (e == hipSuccess) e = launch_cg_finish_cols(states, w.partials, tiles, n, kFinishAlpha, s);
            if (e == hipSuccess) e = launch_hop(k3, s);
            if (e == hipSuccess) e = launch_hop(k4, s, &tiles);
            hop_launches += 4;
        }
        if (e == hipSuccess) e = launch_cg_finish_cols(states, w.partials, tiles, n, kFinishBeta, s);
        if (e == hipSuccess) e = launch_xpay_cols(vs, w.p, w.r, x, fs, n, states, s);
        return e;
    };

    for (;;) {
        bool any = false;
        for (int k = 0; k < n; ++k) any = any || active[k];
        if (!any) break;
        // iterate until every active column has stopped
        for (;;) {
            for (int q = 0; q < check; ++q) TRY(iteration());
            TRY(read_states());
            bool running = false;
            for (int k = 0; k < n; ++k) running = running || (active[k] && hs[k].done == kDoneRunning);
            if (!running) break;
        }
        // FP64 true residuals; restart the columns above tolerance
        TRY(true_residuals());
        TRY(read_states());
        for (int k = 0; k < n; ++k) {
            if (!active[k]) continue;
            const double rr_true = hs[k].result[0];
            stats[k].iters = hs[k].iter;
            stats[k].reliable_updates += 1;
            stats[k].iter_rel_residual = std::sqrt(hs[k].rr / bnorm[k]);
            stats[k].true_rel_residual = std::sqrt(rr_true / bnorm[k]);
            if (rr_true <= o.tol * o.tol * bnorm[k]) {
                stats[k].converged = 1;
                active[k] = 0;
                continue;
            }
            if (!std::isfinite(rr_true) || hs[k].done == kDoneBreakdown) {
                status = TMQCD_EBREAKDOWN;
                active[k] = 0;
                continue;
            }
            if (hs[k].iter >= o.max_iter) {
                if (status == TMQCD_OK) status = TMQCD_ENOCONV;
                active[k] = 0;
                continue;
            }
            StateInit v = none();
            v.set_beta = v.set_done = v.set_rr = true;
            v.beta = rr_true / (hs[k].rr_prev > 0 ? hs[k].rr_prev : rr_true);
            v.rr = rr_true;
            v.done = kDoneRunning;
            TRY(launch_set_state(states + k, v, s));
            TRY(launch_xpay(vs, w.p + k * fs, TMQCD_F64, w.r + k * fs, TMQCD_F64, states + k, false, s));
        }
        // finished columns keep done != 0, so the launches skip them
        for (int k = 0; k < n; ++k)
            if (!active[k]) {
                StateInit v = none();
                v.set_done = true;
                v.done = hs[k].done == kDoneBreakdown ? kDoneBreakdown : kDoneStop;
                TRY(launch_set_state(states + k, v, s));
            }
    }
    TRY(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    const int per_apply = full ? 2 : 4;
    for (int k = 0; k < n; ++k) {
        stats[k].hop_launches = hop_launches + per_apply * applies;
        stats[k].seconds = secs;
    }
    return status;
}

#undef TRY

}  // namespace tmqcd
