// Operator composition (M, M^+, Mhat, Mhat^+, their normal operators) and the
// CG solvers built on the hop kernel.
//
// Even-odd preconditioning (paper, section 2.1): the Schur complement on even
// sites Mhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe, with A = 1 + i w gamma5,
// w = 2 kappa mu.  In the chiral basis gamma5 = diag(-1,-1,+1,+1), so A acts on
// the upper two spins as (1 - i w) and on the lower two as (1 + i w).  The
// adjoints use H^+ (gamma_mu -> -gamma_mu) and A^+ = A(-mu).
//
// One CG iteration on Mhat^+ Mhat is four hop launches and one BLAS launch:
//   t1 = A^{-1} H_oe p                         its block 0 first finishes the
//                                               previous iteration's |r|^2, beta
//                                               and stop tests (when pending)
//   t2 = A p - kappa^2 H_eo t1                 and per-block sums of |t2|^2
//   t3 = A(-mu)^{-1} H^+_oe t2                 its block 0 first finishes
//                                               p^+ A p = |t2|^2 and alpha
//   (A p) = A(-mu) t2 - kappa^2 H^+_eo t3      fused with r -= alpha A p and
//                                               per-block |r|^2
//   x += alpha p, p = r + beta p               every block forms beta itself
//                                               from those partials (the same
//                                               fixed order in every block);
//                                               x here, not in the update hop,
//                                               saves one read of p
// and the host reads the state after a one-block finish of the last beta.
// The reductions finish in a later launch: a last-block-done scheme would
// need a device-wide release in every block, which on this chip writes back
// the XCD's L2 and costs more than a launch.
// All scalars stay on the device; the host queues several iterations, then
// reads the state once.  Kernels queued after convergence return at once.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "device.h"
#include "internal.h"
#include "ops.h"

namespace tmqcd {

thread_local int g_last_hip_error = 0;

namespace {

Cplx cx(double re, double im) { return {re, im}; }
Cplx cdiv1(Cplx z) {   // 1 / z
    const double d = z.re * z.re + z.im * z.im;
    return {z.re / d, -z.im / d};
}

}  // namespace

OpCtx make_ctx(const tmqcd_problem& prob, int prec, int recon, const void* gauge, hipStream_t s) {
    OpCtx c;
    c.g = make_geom(prob);
    c.prec = prec;
    c.recon = recon;
    c.gauge = gauge;
    c.s = s;
    c.kappa = prob.kappa;
    c.w = 2.0 * prob.kappa * prob.mu;
    for (int i = 0; i < 4; ++i) c.bc[i] = {prob.bc[i][0], prob.bc[i][1]};
    return c;
}

// A(+mu) or A(-mu) = A^+, upper/lower chiral halves
static void twist(const OpCtx& c, bool dag, Cplx& up, Cplx& dn) {
    const double w = dag ? -c.w : c.w;
    up = cx(1.0, -w);
    dn = cx(1.0, w);
}

static HopParams base_params(const OpCtx& c) {
    HopParams a;
    std::memset(&a, 0, sizeof(a));
    a.g = c.g;
    a.prec = c.prec;
    a.recon = c.recon;
    a.gauge = c.gauge;
    for (int i = 0; i < 4; ++i) a.bc[i] = c.bc[i];
    a.epi = kEpiStore;
    a.vprec = c.prec == TMQCD_F64 ? TMQCD_F64 : TMQCD_F32;
    return a;
}

static void set_rhs(HopParams& a, const Rhs& r) {
    a.nrhs = r.n;
    a.in_fstride = r.in;
    a.own_fstride = r.own;
    a.out_fstride = r.out;
}

hipError_t op_dslash_pq(const OpCtx& c, const void* in, void* out, int out_parity, double coef, const Rhs& r = kOne) {
    HopParams a = base_params(c);
    a.in = in;
    a.out = out;
    a.out_parity = out_parity;
    a.nparity = 1;
    a.cu_hop = a.cd_hop = cx(coef, 0);
    set_rhs(a, r);
    return launch_hop(a, c.s);
}

// full field: out = A(+-mu) in - kappa H(^+) in
HopParams hp_full(const OpCtx& c, const void* in, void* out, bool dag, int epi, CgState* st, double* partials,
                         void* x, void* r, const void* p, const Rhs& rh) {
    HopParams a = base_params(c);
    a.in = in;
    a.own = in;
    a.out = out;
    a.nparity = 2;
    a.dag = dag;
    twist(c, dag, a.cu_own, a.cd_own);
    a.cu_hop = a.cd_hop = cx(-c.kappa, 0);
    a.epi = epi;
    a.st = st;
    a.partials = partials;
    a.x = x;
    a.r = r;
    a.p = p;
    set_rhs(a, Rhs{rh.n, rh.in, rh.in, rh.out});
    return a;
}
hipError_t op_full(const OpCtx& c, const void* in, void* out, bool dag, int epi, CgState* st, double* partials,
                   void* x, void* r, const void* p, const Rhs& rh = kOne) {
    return launch_hop(hp_full(c, in, out, dag, epi, st, partials, x, r, p, rh), c.s);
}

// even sites: t_o = A(+-mu)^{-1} H(^+)_oe in_e
HopParams hp_schur_first(const OpCtx& c, const void* in_e, void* t_o, bool dag, const Rhs& r) {
    HopParams a = base_params(c);
    a.in = in_e;
    a.out = t_o;
    a.out_parity = 1;
    a.nparity = 1;
    a.dag = dag;
    Cplx up, dn;
    twist(c, dag, up, dn);
    a.cu_hop = cdiv1(up);
    a.cd_hop = cdiv1(dn);
    set_rhs(a, r);
    return a;
}
hipError_t op_schur_first(const OpCtx& c, const void* in_e, void* t_o, bool dag, const Rhs& r = kOne) {
    return launch_hop(hp_schur_first(c, in_e, t_o, dag, r), c.s);
}

// even sites: out_e = A(+-mu) own_e - kappa^2 H(^+)_eo t_o
HopParams hp_schur_second(const OpCtx& c, const void* t_o, const void* own_e, void* out_e, bool dag, int epi,
                          CgState* st, double* partials, void* x, void* r, const void* p, const Rhs& rh) {
    HopParams a = base_params(c);
    a.in = t_o;
    a.own = own_e;
    a.out = out_e;
    a.out_parity = 0;
    a.nparity = 1;
    a.dag = dag;
    twist(c, dag, a.cu_own, a.cd_own);
    a.cu_hop = a.cd_hop = cx(-c.kappa * c.kappa, 0);
    a.epi = epi;
    a.st = st;
    a.partials = partials;
    a.x = x;
    a.r = r;
    a.p = p;
    set_rhs(a, rh);
    return a;
}
hipError_t op_schur_second(const OpCtx& c, const void* t_o, const void* own_e, void* out_e, bool dag, int epi,
                           CgState* st, double* partials, void* x, void* r, const void* p, const Rhs& rh = kOne) {
    return launch_hop(hp_schur_second(c, t_o, own_e, out_e, dag, epi, st, partials, x, r, p, rh), c.s);
}

static int in_subset_of(int op) {
    if (op == TMQCD_DSLASH_EO) return TMQCD_ODD;
    if (op == TMQCD_M || op == TMQCD_MDAG || op == TMQCD_MDAGM) return TMQCD_FULL;
    return TMQCD_EVEN;
}
static int out_subset_of(int op) {
    if (op == TMQCD_DSLASH_OE) return TMQCD_ODD;
    if (op == TMQCD_M || op == TMQCD_MDAG || op == TMQCD_MDAGM) return TMQCD_FULL;
    return TMQCD_EVEN;
}

// out = op(in) for nrhs fields; temporaries from tmp (dslash_tmp_bytes(g, op, prec) * nrhs bytes)
hipError_t apply_operator(const OpCtx& c, int op, const void* in, void* out, char* tmp, int nrhs) {
    const int64_t hb = half_field_bytes(c.g, c.prec);
    const int64_t fi = field_bytes(c.g, c.prec, in_subset_of(op)), fo = field_bytes(c.g, c.prec, out_subset_of(op));
    const Rhs io{nrhs, fi, fi, fo};
    hipError_t e = hipSuccess;
    switch (op) {
        case TMQCD_DSLASH_EO: return op_dslash_pq(c, in, out, 0, -c.kappa, io);
        case TMQCD_DSLASH_OE: return op_dslash_pq(c, in, out, 1, -c.kappa, io);
        case TMQCD_M: return op_full(c, in, out, false, kEpiStore, nullptr, nullptr, nullptr, nullptr, nullptr, io);
        case TMQCD_MDAG: return op_full(c, in, out, true, kEpiStore, nullptr, nullptr, nullptr, nullptr, nullptr, io);
        case TMQCD_MDAGM: {
            const Rhs first{nrhs, fi, fi, 2 * hb}, second{nrhs, 2 * hb, 2 * hb, fo};
            e = op_full(c, in, tmp, false, kEpiStore, nullptr, nullptr, nullptr, nullptr, nullptr, first);
            if (e != hipSuccess) return e;
            return op_full(c, tmp, out, true, kEpiStore, nullptr, nullptr, nullptr, nullptr, nullptr, second);
        }
        case TMQCD_MHAT:
        case TMQCD_MHATDAG: {
            const bool dag = op == TMQCD_MHATDAG;
            e = op_schur_first(c, in, tmp, dag, Rhs{nrhs, fi, 0, hb});
            if (e != hipSuccess) return e;
            return op_schur_second(c, tmp, in, out, dag, kEpiStore, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   Rhs{nrhs, hb, fi, fo});
        }
        case TMQCD_MHATDAGMHAT: {
            char* t_o = tmp;
            char* t_e = tmp + nrhs * hb;
            e = op_schur_first(c, in, t_o, false, Rhs{nrhs, fi, 0, hb});
            if (e != hipSuccess) return e;
            e = op_schur_second(c, t_o, in, t_e, false, kEpiStore, nullptr, nullptr, nullptr, nullptr, nullptr,
                                Rhs{nrhs, hb, fi, hb});
            if (e != hipSuccess) return e;
            e = op_schur_first(c, t_e, t_o, true, Rhs{nrhs, hb, 0, hb});
            if (e != hipSuccess) return e;
            return op_schur_second(c, t_o, t_e, out, true, kEpiStore, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   Rhs{nrhs, hb, hb, fo});
        }
    }
    return hipErrorInvalidValue;
}

int64_t dslash_tmp_bytes(const Geom& g, int op, int prec) {
    const int64_t hb = half_field_bytes(g, prec);
    switch (op) {
        case TMQCD_MDAGM: return 2 * hb;
        case TMQCD_MHAT:
        case TMQCD_MHATDAG: return hb;
        case TMQCD_MHATDAGMHAT: return 2 * hb;
    }
    return 0;
}

// ------------------------------------------------------ even-odd force ---
// S = phi_e^+ (Mhat^+ Mhat)^{-1} phi_e with X_e = (Mhat^+ Mhat)^{-1} phi_e.  The
// links enter Mhat only through H_eo and H_oe, and differentiating both hops gives
// the full-lattice force formula with
//   X = (X_e, X_o),        X_o = A(mu)^{-1} H_oe X_e,
//   Y = kappa (Y_e, Y_o),  Y_e = Mhat X_e,  Y_o = A(-mu)^{-1} (H^+)_oe Y_e,
// (the paper's force section applied to the Schur complement of its even-odd
// preconditioning).  X_o is the first half of Mhat X_e, so three hops make all
// three fields; the kappa of Y goes into the force's scale.
hipError_t force_eo(const OpCtx& c, const void* X_e, double* out, double scale, int accumulate, char* tmp) {
    const int64_t hb = half_field_bytes(c.g, TMQCD_F64);
    char* x_o = tmp;
    char* y_e = tmp + hb;
    char* y_o = tmp + 2 * hb;
    hipError_t e = op_schur_first(c, X_e, x_o, false);
    if (e != hipSuccess) return e;
    e = op_schur_second(c, x_o, X_e, y_e, false, kEpiStore, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (e != hipSuccess) return e;
    e = op_schur_first(c, y_e, y_o, true);
    if (e != hipSuccess) return e;
    const void* const X[2] = {X_e, x_o};
    const void* const Y[2] = {y_e, y_o};
    return launch_force(c.g, c.gauge, c.recon, X, Y, out, c.bc, c.kappa, scale * c.kappa, accumulate, c.s);
}

int64_t force_eo_tmp_bytes(const Geom& g) { return 3 * half_field_bytes(g, TMQCD_F64); }

// ------------------------------------------------------------- workspace ---
static int64_t align(int64_t v) { return round_up(v, kAlignBytes); }

int64_t state_bytes() { return align(sizeof(CgState)); }
int64_t partial_bytes(const Geom& g) { return align(8 * (int64_t)hop_blocks(g, 2) + 8 * kBlock); }

CgWorkspace carve_cg(const Geom& g, int op, int inner_prec, char* base) {
    CgWorkspace w;
    std::memset(&w, 0, sizeof(w));
    const bool full = op == TMQCD_MDAGM;
    const int nh = full ? 2 : 1;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align(bytes);
        return p;
    };
    w.st = reinterpret_cast<CgState*>(take(sizeof(CgState)));
    w.partials = reinterpret_cast<double*>(take(partial_bytes(g)));
    w.partials_b = reinterpret_cast<double*>(take(partial_bytes(g)));
    const int64_t h64 = half_field_bytes(g, TMQCD_F64);
    w.r = take(nh * h64);
    w.p = take(nh * h64);
    w.ax = take(nh * h64);
    if (full) {
        w.t1 = take(2 * h64);
    } else {
        w.t1 = take(h64);
        w.t2 = take(h64);
        w.t3 = take(h64);
    }
    if (inner_prec != TMQCD_F64) {
        const int pv = TMQCD_F32;
        const int64_t hv = half_field_bytes(g, pv), hd = half_field_bytes(g, inner_prec);
        w.rs = take(nh * hv);
        w.xs = take(nh * hv);
        w.ps = take(nh * hd);
        if (full) {
            w.t1s = take(2 * hd);
        } else {
            w.t1s = take(hd);
            w.t2s = take(hd);
            w.t3s = take(hd);
        }
    }
    w.total = off;
    return w;
}

// ------------------------------------------------------------------ CG ---
namespace {

struct Fields {
    void* x;
    void* r;
    void* p;
    void* t1;
    void* t2;
    void* t3;
};

// Queue one CG iteration (all precisions): see the file header.  Every stage
// carries the solver state, so stages queued after the stop return at once.  The
// alpha reductions use partials_a, the beta reductions partials_b: the first hop
// of an iteration finishes the previous iteration's beta (from partials_b) while
// it writes nothing there.  nb_update: the partial count of the update hop (set
// by the first iteration queued; the first hop of that one has no pending finish).
hipError_t queue_iteration(const OpCtx& c, bool full, const Fields& f, CgState* st, double* partials_a,
                           double* partials_b, int pv, int& nb_update) {
    hipError_t e;
    int nb = 0;
    VecSpec vs{&c.g, full ? 2 : 1};
    if (full) {
        HopParams k1 = hp_full(c, f.p, f.t1, false, kEpiStoreNorm, st, partials_a, nullptr, nullptr, nullptr, kOne);
        k1.fin_partials = partials_b;
        k1.fin_n = nb_update;
        k1.fin_kind = kFinishBetaPending;
        e = launch_hop(k1, c.s, &nb);
        if (e == hipSuccess) e = launch_cg_finish(st, partials_a, nb, kFinishAlpha, c.s);
        if (e == hipSuccess)
            e = launch_hop(hp_full(c, f.t1, nullptr, true, kEpiCgUpdate, st, partials_b, nullptr, f.r, nullptr, kOne),
                           c.s, &nb_update);
    } else {
        HopParams k1 = hp_schur_first(c, f.p, f.t1, false, kOne);
        HopParams k3 = hp_schur_first(c, f.t2, f.t3, true, kOne);
        k1.st = k3.st = st;
        k1.fin_partials = partials_b;
        k1.fin_n = nb_update;
        k1.fin_kind = kFinishBetaPending;
        e = launch_hop(k1, c.s);
        if (e == hipSuccess)
            e = launch_hop(hp_schur_second(c, f.t1, f.p, f.t2, false, kEpiStoreNorm, st, partials_a, nullptr, nullptr,
                                           nullptr, kOne),
                           c.s, &nb);
        // the first block of the next hop finishes p^+ A p and alpha (the update hop after it needs alpha)
        k3.fin_partials = partials_a;
        k3.fin_n = nb;
        k3.fin_kind = kFinishAlpha;
        if (e == hipSuccess) e = launch_hop(k3, c.s);
        if (e == hipSuccess)
            e = launch_hop(hp_schur_second(c, f.t3, f.t2, nullptr, true, kEpiCgUpdate, st, partials_b, nullptr, f.r,
                                           nullptr, kOne),
                           c.s, &nb_update);
    }
    if (e != hipSuccess) return e;
    // x += alpha p and p = r + beta p, beta formed from the update's partials; the state's beta finish is pending
    return launch_xpay_fused(vs, f.p, c.prec, f.r, pv, f.x, st, partials_b, nb_update, c.s);
}

// The pending beta finish of the last iteration queued (before the host reads the state).
hipError_t finish_pending(CgState* st, const double* partials_b, int nb_update, hipStream_t s) {
    return nb_update > 0 ? launch_cg_finish(st, partials_b, nb_update, kFinishBetaPending, s) : hipSuccess;
}

struct HostState {
    CgState s;
};

hipError_t read_state(CgState* st, HostState& h, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(&h.s, st, sizeof(CgState), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

StateInit no_change() {
    StateInit v;
    std::memset(&v, 0, sizeof(v));
    return v;
}

}  // namespace

#define TRY(expr)                                     \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) {                       \
            g_last_hip_error = (int)e_;               \
            return TMQCD_EHIP;                        \
        }                                             \
    } while (0)

// The graph of a batch of iterations and, on the null stream, the stream it runs on; released
// on every return path.
struct IterGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t own = nullptr;
    ~IterGraph() {   // teardown: the solve's status is already decided, so errors here are dropped
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (own) {
            (void)hipStreamSynchronize(own);
            (void)hipStreamDestroy(own);
        }
    }
};
constexpr int kGraphIters = 8;             // iterations per captured graph

int run_cg(const tmqcd_problem& prob, const void* const gauge[3], const void* b, void* x, const tmqcd_cg_opts& o,
           tmqcd_cg_stats& stats, void* ws, hipStream_t s_user) {
    const auto t0 = std::chrono::steady_clock::now();
    std::memset(&stats, 0, sizeof(stats));
    const bool graph = o.use_graph == 1;
    IterGraph ig;
    hipStream_t s = s_user;
    if (graph && s == nullptr) {   // the null stream cannot be captured; a blocking stream orders with it
        TRY(hipStreamCreate(&ig.own));
        s = ig.own;
    }
    const bool full = o.op == TMQCD_MDAGM;
    const int nh = full ? 2 : 1;
    const int q = o.inner_prec;
    const bool mixed = q != TMQCD_F64;
    const Geom g = make_geom(prob);
    CgWorkspace w = carve_cg(g, o.op, q, static_cast<char*>(ws));
    const OpCtx c64 = make_ctx(prob, TMQCD_F64, o.recon, gauge[TMQCD_F64], s);
    const OpCtx cq = mixed ? make_ctx(prob, q, o.recon, gauge[q], s) : c64;
    const VecSpec vs{&g, nh};
    const int op = full ? TMQCD_MDAGM : TMQCD_MHATDAGMHAT;
    const int hops_per_apply = full ? 2 : 4;
    const int check = o.check_every > 0 ? o.check_every : 32;
    // default reliable-update factor per inner precision (measured on 32^3 x 64:
    // fewer FP64 restarts at the same iteration count and final residual)
    const double delta = o.reliable_delta > 0 ? o.reliable_delta : (q == TMQCD_F16 ? 1e-2 : 1e-4);
    char* tmp64 = static_cast<char*>(w.t1);   // t1 (and t2 for even-odd) are contiguous

    // state: iteration count, cap
    StateInit si = no_change();
    si.set_iter = si.set_max_iter = si.set_done = true;
    si.iter = 0;
    si.max_iter = o.max_iter;
    si.done = kDoneRunning;
    TRY(launch_set_state(w.st, si, s));

    // r = b - A x (FP64); |b|^2 -> result[1], |r|^2 -> result[0]
    int applies = 0;
    auto true_residual = [&]() -> hipError_t {
        hipError_t e = apply_operator(c64, op, x, w.ax, tmp64, 1);
        if (e != hipSuccess) return e;
        ++applies;
        return launch_residual(vs, w.r, b, w.ax, w.st, 0, w.partials, s);
    };
    if (o.x_is_zero) {
        TRY(launch_zero(vs, x, TMQCD_F64, s));
        TRY(launch_convert(vs, w.r, TMQCD_F64, b, TMQCD_F64, s));
        TRY(launch_norm2(vs, w.r, TMQCD_F64, w.st, 0, w.partials, s));
    } else {
        TRY(true_residual());
    }
    TRY(launch_norm2(vs, b, TMQCD_F64, w.st, 1, w.partials, s));
    HostState hs;
    TRY(read_state(w.st, hs, s));
    const double bb = hs.s.result[1];
    double rr = hs.s.result[0];
    if (!std::isfinite(rr) || !std::isfinite(bb)) {
        TRY(hipStreamSynchronize(s));
        return TMQCD_EBREAKDOWN;
    }
    if (bb == 0.0) {   // b = 0: x = 0 is exact
        TRY(launch_zero(vs, x, TMQCD_F64, s));
        stats.converged = 1;
        stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        TRY(hipStreamSynchronize(s));
        return TMQCD_OK;
    }
    const double target = o.tol * o.tol * bb;

    int iters_done = 0;
    // fields of the iteration
    Fields f;
    int pv;
    if (mixed) {
        pv = TMQCD_F32;
        f = Fields{w.xs, w.rs, w.ps, w.t1s, w.t2s, w.t3s};
        TRY(launch_convert(vs, w.rs, pv, w.r, TMQCD_F64, s));
        TRY(launch_zero(vs, w.xs, pv, s));
        TRY(launch_convert(vs, w.ps, q, w.r, TMQCD_F64, s));
    } else {
        pv = TMQCD_F64;
        f = Fields{x, w.r, w.p, w.t1, w.t2, w.t3};
        TRY(launch_convert(vs, w.p, TMQCD_F64, w.r, TMQCD_F64, s));
    }
    // A low-precision inner solve may stagnate above its trigger; after
    // kCycleCap iterations it returns to an FP64 update regardless.
    constexpr int kCycleCap = 500;
    auto start_cycle = [&](double rr_now) -> hipError_t {
        StateInit v = no_change();
        v.set_rr = v.set_stop = v.set_done = v.set_cycle_end = true;
        v.rr = rr_now;
        v.stop_rr = mixed ? std::max(delta * delta * rr_now, target) : target;
        v.cycle_end = mixed ? iters_done + kCycleCap : o.max_iter;
        v.done = kDoneRunning;
        return launch_set_state(w.st, v, s);
    };
    TRY(start_cycle(rr));
    int nb_update = 0;   // partials of the update hop (known once an iteration has been queued)
    if (graph) {   // every stage of an iteration queued after the stop returns at once, so replays are safe
        TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t ec = hipSuccess;
        for (int k = 0; k < kGraphIters && ec == hipSuccess; ++k)
            ec = queue_iteration(cq, full, f, w.st, w.partials, w.partials_b, pv, nb_update);
        if (ec == hipSuccess) ec = finish_pending(w.st, w.partials_b, nb_update, s);   // each replay ends finished
        const hipError_t ee = hipStreamEndCapture(s, &ig.graph);
        TRY(ec);
        TRY(ee);
        TRY(hipGraphInstantiate(&ig.exec, ig.graph, nullptr, nullptr, 0));
    }

    int status = TMQCD_OK;
    for (;;) {
        if (rr > target) {
            // Queue iterations in batches until the device flags a stop.  After the
            // first batch, each batch is sized from the observed convergence rate so
            // that few iterations are queued past the stop (those return at once).
            int batch = std::min(check, 8);
            double rr_poll = rr;
            int it_poll = iters_done;
            for (;;) {
                if (graph) {
                    for (int k = 0; k < batch; k += kGraphIters) TRY(hipGraphLaunch(ig.exec, s));
                } else {
                    for (int k = 0; k < batch; ++k)
                        TRY(queue_iteration(cq, full, f, w.st, w.partials, w.partials_b, pv, nb_update));
                    TRY(finish_pending(w.st, w.partials_b, nb_update, s));
                }
                TRY(read_state(w.st, hs, s));
                if (hs.s.done != kDoneRunning) break;
                int next = check;
                const int di = hs.s.iter - it_poll;
                if (di > 0 && hs.s.rr > 0 && hs.s.rr < rr_poll) {
                    const double rate = std::log(hs.s.rr / rr_poll) / di;
                    const double need = std::ceil(std::log(hs.s.stop_rr / hs.s.rr) / rate);
                    next = need < 1 ? 1 : (need > check ? check : (int)need);
                }
                batch = next;
                rr_poll = hs.s.rr;
                it_poll = hs.s.iter;
            }
            iters_done = hs.s.iter;
        }
        // fold the low-precision solution into x and recompute the FP64 residual
        if (mixed) TRY(launch_accumulate(vs, x, w.xs, pv, s));
        TRY(true_residual());
        TRY(read_state(w.st, hs, s));
        const double rr_true = hs.s.result[0];
        stats.reliable_updates += 1;
        stats.iter_rel_residual = std::sqrt(hs.s.rr / bb);
        if (!std::isfinite(rr_true)) {
            status = TMQCD_EBREAKDOWN;
            break;
        }
        if (rr_true <= target) {
            stats.converged = 1;
            rr = rr_true;
            break;
        }
        if (hs.s.done == kDoneBreakdown) {
            status = TMQCD_EBREAKDOWN;
            rr = rr_true;
            break;
        }
        if (hs.s.iter >= o.max_iter) {
            status = TMQCD_ENOCONV;
            rr = rr_true;
            break;
        }
        // reliable update: restart the recursion from the true residual, keeping
        // the search direction: p = r + (rr_true / rr_prev) p
        const double rr_prev = hs.s.rr_prev > 0 ? hs.s.rr_prev : rr_true;
        if (mixed) TRY(launch_convert(vs, w.rs, pv, w.r, TMQCD_F64, s));
        StateInit v = no_change();
        v.set_beta = true;
        v.beta = rr_true / rr_prev;
        v.set_done = true;
        v.done = kDoneRunning;
        TRY(launch_set_state(w.st, v, s));
        TRY(launch_xpay(vs, f.p, cq.prec, f.r, pv, w.st, false, s));
        rr = rr_true;
        TRY(start_cycle(rr));
    }
    stats.iters = iters_done;
    stats.inner_iters = mixed ? iters_done : 0;
    stats.hop_launches = hops_per_apply * (iters_done + applies);
    stats.true_rel_residual = std::sqrt(rr / bb);
    TRY(hipStreamSynchronize(s));
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

#undef TRY

}  // namespace tmqcd
