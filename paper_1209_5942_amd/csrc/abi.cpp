// The C interface: host-side argument validation (no HIP call before every
// argument has been checked), dispatch to the operator and solver code, and
// error reporting.  See include/tmqcd.h for the contract of each entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "device.h"
#include "internal.h"
#include "ops.h"
#include "tmqcd.h"

using namespace tmqcd;

namespace {

bool valid_problem(const tmqcd_problem* p) {
    if (!p) return false;
    int64_t v = 1;
    for (int i = 0; i < 4; ++i) {
        const int d = p->dims[i];
        if (d < 2 || (d & 1)) return false;
        v *= d;
        if (v > (int64_t)1 << 32) return false;   // half volume must fit in int32 site indices
    }
    if (!std::isfinite(p->kappa) || !std::isfinite(p->mu)) return false;
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(p->bc[i][0]) || !std::isfinite(p->bc[i][1])) return false;
    return true;
}
bool valid_prec(int p) { return p == TMQCD_F64 || p == TMQCD_F32 || p == TMQCD_F16; }
bool valid_recon(int r) { return r == TMQCD_RECON18 || r == TMQCD_RECON12 || r == TMQCD_RECON10 || r == TMQCD_RECON8; }
bool valid_subset(int s) { return s == TMQCD_FULL || s == TMQCD_EVEN || s == TMQCD_ODD; }
bool valid_op(int op) { return op >= TMQCD_DSLASH_EO && op <= TMQCD_MHATDAGMHAT; }
bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
bool overlap(const void* a, int64_t na, const void* b, int64_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + (uintptr_t)nb && y < x + (uintptr_t)na;
}

int in_subset(int op) {
    switch (op) {
        case TMQCD_DSLASH_EO: return TMQCD_ODD;
        case TMQCD_DSLASH_OE: return TMQCD_EVEN;
        case TMQCD_M:
        case TMQCD_MDAG:
        case TMQCD_MDAGM: return TMQCD_FULL;
    }
    return TMQCD_EVEN;
}
int out_subset(int op) {
    switch (op) {
        case TMQCD_DSLASH_EO: return TMQCD_EVEN;
        case TMQCD_DSLASH_OE: return TMQCD_ODD;
        case TMQCD_M:
        case TMQCD_MDAG:
        case TMQCD_MDAGM: return TMQCD_FULL;
    }
    return TMQCD_EVEN;
}

int64_t mom_bytes(const Geom& g) { return 2 * g.vh * 4 * 8 * 8; }

int hip_fail(hipError_t e) {
    g_last_hip_error = (int)e;
    return TMQCD_EHIP;
}

int64_t cg_workspace(const Geom& g, int op, int prec_mask, int nrhs) {
    if (nrhs > 1) return carve_cg_mrhs(g, op, nrhs, nullptr).total;   // FP64 multi-RHS solve
    int64_t need = carve_cg(g, op, TMQCD_F64, nullptr).total;
    if (prec_mask & (1 << TMQCD_F32)) {
        const int64_t t = carve_cg(g, op, TMQCD_F32, nullptr).total;
        need = t > need ? t : need;
    }
    if (prec_mask & (1 << TMQCD_F16)) {
        const int64_t t = carve_cg(g, op, TMQCD_F16, nullptr).total;
        need = t > need ? t : need;
    }
    return need;
}

int64_t dslash_workspace(const Geom& g, int op, int prec_mask, int nrhs) {
    int64_t need = 0;
    for (int p = 0; p < 3; ++p)
        if (prec_mask & (1 << p)) {
            const int64_t t = nrhs * dslash_tmp_bytes(g, op, p);
            need = t > need ? t : need;
        }
    return need;
}

}  // namespace

extern "C" {

size_t tmqcd_gauge_bytes(const tmqcd_problem* prob, int prec, int recon) {
    if (!valid_problem(prob) || !valid_prec(prec) || !valid_recon(recon)) return 0;
    return (size_t)gauge_bytes(make_geom(*prob), prec, recon);
}

size_t tmqcd_spinor_bytes(const tmqcd_problem* prob, int prec, int subset, int nrhs) {
    if (!valid_problem(prob) || !valid_prec(prec) || !valid_subset(subset) || nrhs < 1 || nrhs > kMaxRhs) return 0;
    return (size_t)(nrhs * field_bytes(make_geom(*prob), prec, subset));
}

size_t tmqcd_workspace_bytes(const tmqcd_problem* prob, int op, int prec_mask, int nrhs) {
    if (!valid_problem(prob) || nrhs < 1 || nrhs > kMaxRhs) return 0;
    if (op == -1) return (size_t)round_up(8 * aux_partials_doubles(make_geom(*prob)), kAlignBytes);
    if (!valid_op(op) || (prec_mask & ~7) || prec_mask == 0) return 0;
    const Geom g = make_geom(*prob);
    int64_t need = dslash_workspace(g, op, prec_mask, nrhs);
    if (op == TMQCD_MDAGM || op == TMQCD_MHATDAGMHAT) {
        const int64_t t = cg_workspace(g, op, prec_mask, nrhs);
        need = t > need ? t : need;
    }
    return (size_t)(need > 256 ? need : 256);
}

int tmqcd_pack_gauge(const tmqcd_problem* prob, const void* U_canon, void* U_packed, int prec, int recon,
                     void* stream) {
    if (!valid_problem(prob) || !valid_prec(prec) || !valid_recon(recon) || !U_canon || !U_packed) return TMQCD_EINVAL;
    if (!aligned(U_canon, 16) || !aligned(U_packed, kAlignBytes)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    if (overlap(U_canon, 2 * g.vh * 4 * 9 * 16, U_packed, gauge_bytes(g, prec, recon))) return TMQCD_EALIAS;
    const hipError_t e = launch_pack_gauge(g, U_canon, U_packed, prec, recon, (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_unpack_gauge(const tmqcd_problem* prob, const void* U_packed, void* U_canon, int prec, int recon,
                       void* stream) {
    if (!valid_problem(prob) || !valid_prec(prec) || !valid_recon(recon) || !U_canon || !U_packed) return TMQCD_EINVAL;
    if (!aligned(U_canon, 16) || !aligned(U_packed, kAlignBytes)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    if (overlap(U_canon, 2 * g.vh * 4 * 9 * 16, U_packed, gauge_bytes(g, prec, recon))) return TMQCD_EALIAS;
    const hipError_t e = launch_unpack_gauge(g, U_packed, U_canon, prec, recon, (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

static int pack_common(const tmqcd_problem* prob, const void* canon, const void* packed, int prec, int subset,
                       int nrhs) {
    if (!valid_problem(prob) || !valid_prec(prec) || !valid_subset(subset) || nrhs < 1 || nrhs > kMaxRhs || !canon ||
        !packed)
        return TMQCD_EINVAL;
    if (!aligned(canon, 16) || !aligned(packed, kAlignBytes)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int64_t n = subset == TMQCD_FULL ? 2 * g.vh : g.vh;
    if (overlap(canon, nrhs * n * 12 * 16, packed, nrhs * field_bytes(g, prec, subset))) return TMQCD_EALIAS;
    return TMQCD_OK;
}

int tmqcd_pack_spinor(const tmqcd_problem* prob, const void* in_canon, void* out_packed, int prec, int subset,
                      int nrhs, void* stream) {
    const int rc = pack_common(prob, in_canon, out_packed, prec, subset, nrhs);
    if (rc != TMQCD_OK) return rc;
    const hipError_t e =
        launch_pack_spinor(make_geom(*prob), in_canon, out_packed, prec, subset, nrhs, false, (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_unpack_spinor(const tmqcd_problem* prob, const void* in_packed, void* out_canon, int prec, int subset,
                        int nrhs, void* stream) {
    const int rc = pack_common(prob, out_canon, in_packed, prec, subset, nrhs);
    if (rc != TMQCD_OK) return rc;
    const hipError_t e =
        launch_pack_spinor(make_geom(*prob), out_canon, const_cast<void*>(in_packed), prec, subset, nrhs, true,
                           (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_dslash(const tmqcd_problem* prob, const void* U_packed, const void* in, void* out, int op, int prec,
                 int recon, int nrhs, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_problem(prob) || !valid_op(op) || !valid_prec(prec) || !valid_recon(recon) || nrhs < 1 ||
        nrhs > kMaxRhs || !U_packed || !in || !out)
        return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes) || !aligned(in, kAlignBytes) || !aligned(out, kAlignBytes))
        return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int64_t fin = field_bytes(g, prec, in_subset(op)), fout = field_bytes(g, prec, out_subset(op));
    if (overlap(in, nrhs * fin, out, nrhs * fout)) return TMQCD_EALIAS;
    const int64_t need = nrhs * dslash_tmp_bytes(g, op, prec);
    if (need > 0) {
        if (!ws || (int64_t)ws_bytes < need) return TMQCD_EWORKSPACE;
        if (!aligned(ws, kAlignBytes)) return TMQCD_EALIGN;
        if (overlap(ws, need, in, nrhs * fin) || overlap(ws, need, out, nrhs * fout)) return TMQCD_EALIAS;
    }
    const OpCtx c = make_ctx(*prob, prec, recon, U_packed, (hipStream_t)stream);
    const hipError_t e = apply_operator(c, op, in, out, static_cast<char*>(ws), nrhs);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

size_t tmqcd_bicgstab_workspace_bytes(const tmqcd_problem* prob, int op) {
    if (!valid_problem(prob) || (op != TMQCD_M && op != TMQCD_MHAT)) return 0;
    return (size_t)bicgstab_workspace(make_geom(*prob), op);
}

int tmqcd_bicgstab(const tmqcd_problem* prob, const void* U_packed, const void* b, void* x,
                   const tmqcd_cg_opts* opts, tmqcd_cg_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_problem(prob) || !U_packed || !b || !x || !opts || !stats) return TMQCD_EINVAL;
    const tmqcd_cg_opts& o = *opts;
    if (o.op != TMQCD_M && o.op != TMQCD_MHAT) return TMQCD_EINVAL;
    if (o.inner_prec != TMQCD_F64 || !valid_recon(o.recon) || o.max_iter < 1) return TMQCD_EINVAL;
    if (!(o.tol > 0.0) || !std::isfinite(o.tol) || o.check_every < 0) return TMQCD_EINVAL;
    if (!aligned(b, kAlignBytes) || !aligned(x, kAlignBytes) || !aligned(U_packed, kAlignBytes)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int64_t fb = field_bytes(g, TMQCD_F64, o.op == TMQCD_M ? TMQCD_FULL : TMQCD_EVEN);
    if (overlap(b, fb, x, fb)) return TMQCD_EALIAS;
    const int64_t need = bicgstab_workspace(g, o.op);
    if (!ws || (int64_t)ws_bytes < need) return TMQCD_EWORKSPACE;
    if (!aligned(ws, kAlignBytes)) return TMQCD_EALIGN;
    if (overlap(ws, need, b, fb) || overlap(ws, need, x, fb) ||
        overlap(ws, need, U_packed, gauge_bytes(g, TMQCD_F64, o.recon)))
        return TMQCD_EALIAS;
    return run_bicgstab(*prob, U_packed, b, x, o, *stats, ws, (hipStream_t)stream);
}

int tmqcd_cg(const tmqcd_problem* prob, const void* const U_packed[3], const void* b, void* x,
             const tmqcd_cg_opts* opts, tmqcd_cg_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_problem(prob) || !U_packed || !b || !x || !opts || !stats) return TMQCD_EINVAL;
    const tmqcd_cg_opts& o = *opts;
    if (o.op != TMQCD_MDAGM && o.op != TMQCD_MHATDAGMHAT) return TMQCD_EINVAL;
    if (!valid_prec(o.inner_prec) || !valid_recon(o.recon) || o.max_iter < 1) return TMQCD_EINVAL;
    if (!(o.tol > 0.0) || !std::isfinite(o.tol) || o.reliable_delta < 0 || o.reliable_delta >= 1 ||
        o.check_every < 0 || o.use_graph < -1 || o.use_graph > 1 || o.nrhs < 0 || o.nrhs > kMaxRhs)
        return TMQCD_EINVAL;
    const int nrhs = o.nrhs > 1 ? o.nrhs : 1;
    if (nrhs > 1 && (o.inner_prec != TMQCD_F64 || o.use_graph == 1)) return TMQCD_EINVAL;
    if (!U_packed[TMQCD_F64] || !U_packed[o.inner_prec]) return TMQCD_EINVAL;
    if (!aligned(b, kAlignBytes) || !aligned(x, kAlignBytes) || !aligned(U_packed[TMQCD_F64], kAlignBytes) ||
        !aligned(U_packed[o.inner_prec], kAlignBytes))
        return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int subset = o.op == TMQCD_MDAGM ? TMQCD_FULL : TMQCD_EVEN;
    const int64_t fb = nrhs * field_bytes(g, TMQCD_F64, subset);
    if (overlap(b, fb, x, fb)) return TMQCD_EALIAS;
    const int64_t need = nrhs > 1 ? carve_cg_mrhs(g, o.op, nrhs, nullptr).total
                                  : carve_cg(g, o.op, o.inner_prec, nullptr).total;
    if (!ws || (int64_t)ws_bytes < need) return TMQCD_EWORKSPACE;
    if (!aligned(ws, kAlignBytes)) return TMQCD_EALIGN;
    if (overlap(ws, need, b, fb) || overlap(ws, need, x, fb)) return TMQCD_EALIAS;
    if (nrhs > 1) return run_cg_mrhs(*prob, U_packed[TMQCD_F64], b, x, o, stats, ws, (hipStream_t)stream);
    return run_cg(*prob, U_packed, b, x, o, *stats, ws, (hipStream_t)stream);
}

size_t tmqcd_cg_batch_workspace_bytes(int n, const tmqcd_problem* probs) {
    if (n < 1 || n > 8 || !probs) return 0;
    for (int i = 0; i < n; ++i)
        if (!valid_problem(&probs[i])) return 0;
    return (size_t)cg_batch_workspace(n, probs);
}

int tmqcd_cg_batch(int n, const tmqcd_problem* probs, const void* const* U_packed, const void* const* b,
                   void* const* x, const tmqcd_cg_opts* opts, tmqcd_cg_stats* stats, int use_graph, void* ws,
                   size_t ws_bytes, void* stream) {
    if (n < 1 || n > 8 || !probs || !U_packed || !b || !x || !opts || !stats || (use_graph != 0 && use_graph != 1))
        return TMQCD_EINVAL;
    const tmqcd_cg_opts& o = *opts;
    if (o.op != TMQCD_MHATDAGMHAT || o.inner_prec != TMQCD_F64 || !valid_recon(o.recon) || o.max_iter < 1 ||
        !(o.tol > 0.0) || !std::isfinite(o.tol) || o.check_every < 0)
        return TMQCD_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!valid_problem(&probs[i]) || !U_packed[i] || !b[i] || !x[i]) return TMQCD_EINVAL;
        if (!aligned(U_packed[i], kAlignBytes) || !aligned(b[i], kAlignBytes) || !aligned(x[i], kAlignBytes))
            return TMQCD_EALIGN;
    }
    const int64_t need = cg_batch_workspace(n, probs);
    if (!ws || (int64_t)ws_bytes < need) return TMQCD_EWORKSPACE;
    if (!aligned(ws, kAlignBytes)) return TMQCD_EALIGN;
    for (int i = 0; i < n; ++i) {
        const int64_t fi = field_bytes(make_geom(probs[i]), TMQCD_F64, TMQCD_EVEN);
        if (overlap(ws, need, x[i], fi) || overlap(ws, need, b[i], fi)) return TMQCD_EALIAS;
        for (int j = 0; j < n; ++j) {
            const int64_t fj = field_bytes(make_geom(probs[j]), TMQCD_F64, TMQCD_EVEN);
            if (overlap(x[i], fi, b[j], fj) || (i != j && overlap(x[i], fi, x[j], fj))) return TMQCD_EALIAS;
        }
    }
    return run_cg_batch(n, probs, U_packed, b, x, o, stats, use_graph == 1, ws, (hipStream_t)stream);
}

size_t tmqcd_force_workspace_bytes(const tmqcd_problem* prob) {
    if (!valid_problem(prob)) return 0;
    return (size_t)field_bytes(make_geom(*prob), TMQCD_F64, TMQCD_FULL);
}

int tmqcd_force(const tmqcd_problem* prob, const void* U_packed, int recon, const void* X, const void* Y,
                double* dSdw, double scale, int accumulate, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_problem(prob) || !valid_recon(recon) || !U_packed || !X || !dSdw || !std::isfinite(scale) ||
        (accumulate != 0 && accumulate != 1))
        return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes) || !aligned(X, kAlignBytes) || (Y && !aligned(Y, kAlignBytes)) ||
        !aligned(dSdw, 16))
        return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int64_t fb = field_bytes(g, TMQCD_F64, TMQCD_FULL), ob = mom_bytes(g), gb = gauge_bytes(g, TMQCD_F64, recon);
    if (overlap(dSdw, ob, X, fb) || (Y && overlap(dSdw, ob, Y, fb)) || overlap(dSdw, ob, U_packed, gb))
        return TMQCD_EALIAS;
    if (!Y) {   // Y = M X is computed into the workspace
        if (!ws || (int64_t)ws_bytes < fb) return TMQCD_EWORKSPACE;
        if (!aligned(ws, kAlignBytes)) return TMQCD_EALIGN;
        if (overlap(ws, fb, X, fb) || overlap(ws, fb, U_packed, gb) || overlap(ws, fb, dSdw, ob)) return TMQCD_EALIAS;
    }
    const hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (!Y) {
        const OpCtx c = make_ctx(*prob, TMQCD_F64, recon, U_packed, s);
        e = apply_operator(c, TMQCD_M, X, ws, nullptr, 1);
        if (e != hipSuccess) return hip_fail(e);
        Y = ws;
    }
    Cplx bc[4];
    for (int i = 0; i < 4; ++i) bc[i] = {prob->bc[i][0], prob->bc[i][1]};
    const int64_t hb = half_field_bytes(g, TMQCD_F64);
    const void* const Xp[2] = {X, static_cast<const char*>(X) + hb};
    const void* const Yp[2] = {Y, static_cast<const char*>(Y) + hb};
    e = launch_force(g, U_packed, recon, Xp, Yp, dSdw, bc, prob->kappa, scale, accumulate, s);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

size_t tmqcd_force_eo_workspace_bytes(const tmqcd_problem* prob) {
    if (!valid_problem(prob)) return 0;
    return (size_t)force_eo_tmp_bytes(make_geom(*prob));
}

int tmqcd_force_eo(const tmqcd_problem* prob, const void* U_packed, int recon, const void* X_e, double* dSdw,
                   double scale, int accumulate, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_problem(prob) || !valid_recon(recon) || !U_packed || !X_e || !dSdw || !std::isfinite(scale) ||
        (accumulate != 0 && accumulate != 1))
        return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes) || !aligned(X_e, kAlignBytes) || !aligned(dSdw, 16)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int64_t need = force_eo_tmp_bytes(g);
    if (!ws || (int64_t)ws_bytes < need) return TMQCD_EWORKSPACE;
    if (!aligned(ws, kAlignBytes)) return TMQCD_EALIGN;
    const int64_t fe = field_bytes(g, TMQCD_F64, TMQCD_EVEN), ob = mom_bytes(g),
                  gb = gauge_bytes(g, TMQCD_F64, recon);
    if (overlap(dSdw, ob, X_e, fe) || overlap(dSdw, ob, U_packed, gb) || overlap(dSdw, ob, ws, need) ||
        overlap(ws, need, X_e, fe) || overlap(ws, need, U_packed, gb))
        return TMQCD_EALIAS;
    const OpCtx c = make_ctx(*prob, TMQCD_F64, recon, U_packed, (hipStream_t)stream);
    const hipError_t e = force_eo(c, X_e, dSdw, scale, accumulate, static_cast<char*>(ws));
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_gauge_force(const tmqcd_problem* prob, const void* U_packed, double beta, double* dSdw, double scale,
                      int accumulate, void* stream) {
    if (!valid_problem(prob) || !U_packed || !dSdw || !std::isfinite(beta) || !std::isfinite(scale) ||
        (accumulate != 0 && accumulate != 1))
        return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes) || !aligned(dSdw, 16)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    if (overlap(dSdw, mom_bytes(g), U_packed, gauge_bytes(g, TMQCD_F64, TMQCD_RECON18))) return TMQCD_EALIAS;
    const hipError_t e = launch_gauge_force(g, U_packed, beta, dSdw, scale, accumulate, (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

size_t tmqcd_gauge_force_tlsym_workspace_bytes(const tmqcd_problem* prob) {
    if (!valid_problem(prob)) return 0;
    return (size_t)round_up(staple_field_bytes(make_geom(*prob)), kAlignBytes);
}

int tmqcd_gauge_force_tlsym(const tmqcd_problem* prob, const void* U_packed, double beta, double c1, double* dSdw,
                            double scale, int accumulate, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_problem(prob) || !U_packed || !dSdw || !std::isfinite(beta) || !std::isfinite(c1) ||
        !std::isfinite(scale) || (accumulate != 0 && accumulate != 1))
        return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes) || !aligned(dSdw, 16)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int64_t ub = gauge_bytes(g, TMQCD_F64, TMQCD_RECON18), ob = mom_bytes(g);
    if (overlap(dSdw, ob, U_packed, ub)) return TMQCD_EALIAS;
    if (c1 != 0.0) {
        const int64_t need = staple_field_bytes(g);
        if (!ws || (int64_t)ws_bytes < need) return TMQCD_EWORKSPACE;
        if (!aligned(ws, kAlignBytes)) return TMQCD_EALIGN;
        if (overlap(ws, need, U_packed, ub) || overlap(ws, need, dSdw, ob)) return TMQCD_EALIAS;
    }
    const hipError_t e =
        launch_gauge_force_sym(g, U_packed, beta, c1, dSdw, scale, accumulate, ws, (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_heatbath(const tmqcd_problem* prob, void* U_packed, int prec, double beta, uint64_t seed, uint32_t sweep,
                   void* stream) {
    if (!valid_problem(prob) || !U_packed || (prec != TMQCD_F64 && prec != TMQCD_F32) || !std::isfinite(beta) ||
        beta < 0.0)
        return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    if (4 * 2 * g.vh > 0xFFFFFFFFll) return TMQCD_EINVAL;   // generator counters are 32-bit link ids
    const hipError_t e = launch_su3_sweep(g, U_packed, prec, beta, seed, sweep, true, (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_overrelax(const tmqcd_problem* prob, void* U_packed, int prec, void* stream) {
    if (!valid_problem(prob) || !U_packed || (prec != TMQCD_F64 && prec != TMQCD_F32)) return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes)) return TMQCD_EALIGN;
    const hipError_t e = launch_su3_sweep(make_geom(*prob), U_packed, prec, 0.0, 0, 0, false, (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_update_links(const tmqcd_problem* prob, void* U_packed, const double* p, double dt, void* stream) {
    if (!valid_problem(prob) || !U_packed || !p || !std::isfinite(dt)) return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes) || !aligned(p, 16)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    if (overlap(p, mom_bytes(g), U_packed, gauge_bytes(g, TMQCD_F64, TMQCD_RECON18))) return TMQCD_EALIAS;
    const hipError_t e = launch_update_links(g, U_packed, p, dt, (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

static int aux_ws_check(const Geom& g, void* ws, size_t ws_bytes) {
    if (!ws || (int64_t)ws_bytes < 8 * aux_partials_doubles(g)) return TMQCD_EWORKSPACE;
    if (!aligned(ws, kAlignBytes)) return TMQCD_EALIGN;
    return TMQCD_OK;
}

int tmqcd_plaquette(const tmqcd_problem* prob, const void* U_packed, double* result, void* ws, size_t ws_bytes,
                    void* stream) {
    if (!valid_problem(prob) || !U_packed || !result) return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes) || !aligned(result, 8)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int rc = aux_ws_check(g, ws, ws_bytes);
    if (rc != TMQCD_OK) return rc;
    if (overlap(ws, ws_bytes, U_packed, gauge_bytes(g, TMQCD_F64, TMQCD_RECON18)) || overlap(ws, ws_bytes, result, 8))
        return TMQCD_EALIAS;
    const hipError_t e = launch_plaquette(g, U_packed, result, static_cast<double*>(ws), (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_rectangle(const tmqcd_problem* prob, const void* U_packed, double* result, void* ws, size_t ws_bytes,
                    void* stream) {
    if (!valid_problem(prob) || !U_packed || !result) return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes) || !aligned(result, 8)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int rc = aux_ws_check(g, ws, ws_bytes);
    if (rc != TMQCD_OK) return rc;
    if (overlap(ws, ws_bytes, U_packed, gauge_bytes(g, TMQCD_F64, TMQCD_RECON18)) || overlap(ws, ws_bytes, result, 8))
        return TMQCD_EALIAS;
    const hipError_t e = launch_rectangle(g, U_packed, result, static_cast<double*>(ws), (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_momentum_norm2(const tmqcd_problem* prob, const double* p, double* result, void* ws, size_t ws_bytes,
                         void* stream) {
    if (!valid_problem(prob) || !p || !result) return TMQCD_EINVAL;
    if (!aligned(p, 16) || !aligned(result, 8)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int rc = aux_ws_check(g, ws, ws_bytes);
    if (rc != TMQCD_OK) return rc;
    if (overlap(ws, ws_bytes, p, mom_bytes(g)) || overlap(ws, ws_bytes, result, 8)) return TMQCD_EALIAS;
    const hipError_t e = launch_mom_norm2(g, p, result, static_cast<double*>(ws), (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_delta_h(const tmqcd_problem* prob, const void* U0, const void* U1, const double* p0, const double* p1,
                  const void* phi, const void* X0, const void* X1, int subset, double beta, double c1,
                  double* result, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_problem(prob) || !U0 || !U1 || !p0 || !p1 || !phi || !X0 || !X1 || !result ||
        (subset != TMQCD_FULL && subset != TMQCD_EVEN) || !std::isfinite(beta) || !std::isfinite(c1))
        return TMQCD_EINVAL;
    if (!aligned(U0, kAlignBytes) || !aligned(U1, kAlignBytes) || !aligned(p0, 16) || !aligned(p1, 16) ||
        !aligned(phi, kAlignBytes) || !aligned(X0, kAlignBytes) || !aligned(X1, kAlignBytes) || !aligned(result, 8))
        return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int rc = aux_ws_check(g, ws, ws_bytes);
    if (rc != TMQCD_OK) return rc;
    const int64_t ub = gauge_bytes(g, TMQCD_F64, TMQCD_RECON18), pb = mom_bytes(g), fb = field_bytes(g, TMQCD_F64, subset);
    const void* ins[7] = {U0, U1, p0, p1, phi, X0, X1};
    const int64_t sz[7] = {ub, ub, pb, pb, fb, fb, fb};
    for (int i = 0; i < 7; ++i)
        if (overlap(ws, ws_bytes, ins[i], sz[i]) || overlap(result, 32, ins[i], sz[i])) return TMQCD_EALIAS;
    if (overlap(ws, ws_bytes, result, 32)) return TMQCD_EALIAS;
    const hipError_t e = launch_delta_h(g, U0, U1, p0, p1, phi, X0, X1, subset == TMQCD_FULL ? 2 : 1, beta, c1, result,
                                        static_cast<double*>(ws), (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

int tmqcd_dot(const tmqcd_problem* prob, const void* x, const void* y, int subset, double* result, void* ws,
              size_t ws_bytes, void* stream) {
    if (!valid_problem(prob) || !x || !y || !result || !valid_subset(subset)) return TMQCD_EINVAL;
    if (!aligned(x, kAlignBytes) || !aligned(y, kAlignBytes) || !aligned(result, 8)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int rc = aux_ws_check(g, ws, ws_bytes);
    if (rc != TMQCD_OK) return rc;
    const int64_t fb = field_bytes(g, TMQCD_F64, subset);
    if (overlap(ws, ws_bytes, x, fb) || overlap(ws, ws_bytes, y, fb) || overlap(ws, ws_bytes, result, 16))
        return TMQCD_EALIAS;
    const hipError_t e = launch_spinor_dot(g, x, y, subset == TMQCD_FULL ? 2 : 1, result, static_cast<double*>(ws),
                                           (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

size_t tmqcd_tune_workspace_bytes(const tmqcd_problem* prob, int prec) {
    if (!valid_problem(prob) || !valid_prec(prec)) return 0;
    return (size_t)tune_workspace_bytes(make_geom(*prob), prec);
}

int tmqcd_tune(const tmqcd_problem* prob, const void* U_packed, int prec, int recon, void* ws, size_t ws_bytes,
               tmqcd_tune_result results[3], void* stream) {
    if (!valid_problem(prob) || !valid_prec(prec) || !valid_recon(recon) || !U_packed || !results) return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int64_t need = tune_workspace_bytes(g, prec);
    if (!ws || (int64_t)ws_bytes < need) return TMQCD_EWORKSPACE;
    if (!aligned(ws, kAlignBytes)) return TMQCD_EALIGN;
    if (overlap(ws, need, U_packed, gauge_bytes(g, prec, recon))) return TMQCD_EALIAS;
    return run_tune(*prob, U_packed, prec, recon, ws, (hipStream_t)stream, results);
}

int tmqcd_tune_save(const char* path) { return path ? tune_save(path) : TMQCD_EINVAL; }
int tmqcd_tune_load(const char* path) { return path ? tune_load(path) : TMQCD_EINVAL; }
void tmqcd_tune_clear(void) { tune_clear(); }

int tmqcd_tune_set(const tmqcd_problem* prob, int prec, int recon, int kernel_class, int nrhs, int block,
                   int order, int group) {
    if (!valid_problem(prob) || !valid_prec(prec) || !valid_recon(recon) ||
        !valid_choice(kernel_class, nrhs, block, order, group))
        return TMQCD_EINVAL;
    tune_set(*prob, prec, recon, kernel_class, nrhs, block, order, group);
    return TMQCD_OK;
}

size_t tmqcd_tune_mrhs_workspace_bytes(const tmqcd_problem* prob, int prec, int nrhs) {
    if (!valid_problem(prob) || !valid_prec(prec) || nrhs < 2 || nrhs > kMaxRhs) return 0;
    return (size_t)tune_mrhs_workspace_bytes(make_geom(*prob), prec, nrhs);
}

int tmqcd_tune_mrhs(const tmqcd_problem* prob, const void* U_packed, int prec, int recon, int nrhs, void* ws,
                    size_t ws_bytes, tmqcd_tune_result* result, void* stream) {
    if (!valid_problem(prob) || !valid_prec(prec) || !valid_recon(recon) || nrhs < 2 || nrhs > kMaxRhs ||
        !U_packed || !result)
        return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes)) return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int64_t need = tune_mrhs_workspace_bytes(g, prec, nrhs);
    if (!ws || (int64_t)ws_bytes < need) return TMQCD_EWORKSPACE;
    if (!aligned(ws, kAlignBytes)) return TMQCD_EALIGN;
    if (overlap(ws, need, U_packed, gauge_bytes(g, prec, recon))) return TMQCD_EALIAS;
    return run_tune_mrhs(*prob, U_packed, prec, recon, nrhs, ws, (hipStream_t)stream, result);
}

int tmqcd_hbm_probe(const void* src, void* dst, size_t bytes, int grid, uint32_t* xor_out, void* stream) {
    if (!src || bytes == 0 || bytes % 16 || grid < 1 || grid > 65536 || (!dst && !xor_out)) return TMQCD_EINVAL;
    if (!aligned(src, 16) || (dst && !aligned(dst, 16)) || (!dst && !aligned(xor_out, 4))) return TMQCD_EALIGN;
    if (dst && overlap(src, (int64_t)bytes, dst, (int64_t)bytes)) return TMQCD_EALIAS;
    if (!dst && overlap(src, (int64_t)bytes, xor_out, 4)) return TMQCD_EALIAS;
    const hipError_t e = launch_hbm_probe(src, dst, (int64_t)bytes, grid, reinterpret_cast<unsigned*>(xor_out),
                                          (hipStream_t)stream);
    return e == hipSuccess ? TMQCD_OK : hip_fail(e);
}

const char* tmqcd_error_string(int code) {
    switch (code) {
        case TMQCD_OK: return "success";
        case TMQCD_EINVAL: return "invalid argument (extent, pointer, op, precision, reconstruction or nrhs)";
        case TMQCD_EALIAS: return "output overlaps an input";
        case TMQCD_EALIGN: return "device pointer not aligned (256 bytes for packed fields, 16 for canonical)";
        case TMQCD_ENOCONV: return "CG did not converge within max_iter";
        case TMQCD_EBREAKDOWN: return "CG breakdown (non-finite residual or p^+ A p <= 0)";
        case TMQCD_EHIP: return "HIP runtime error (see tmqcd_last_hip_error)";
        case TMQCD_EWORKSPACE: return "workspace missing or smaller than tmqcd_workspace_bytes";
        case TMQCD_ESCRATCH: return "temporaries larger than the static scratch of tmqcd_dslash_noalloc";
    }
    return "unknown error code";
}

int tmqcd_last_hip_error(void) { return g_last_hip_error; }

}  // extern "C"
