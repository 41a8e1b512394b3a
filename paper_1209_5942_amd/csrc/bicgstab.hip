// BiCGStab on M (full field) or on the even-odd Schur complement Mhat (even
// field), FP64: the paper's second Krylov solver for D phi = psi (§2.1), in
// van der Vorst's form.  Per iteration (rt the shadow residual):
//   p = r + beta (p - omega v);  v = A p;  alpha = rho / (rt, v);  s = r - alpha v;
//   t = A s;  omega = (t, s) / (t, t);  x += alpha p + omega s;  r = s - omega t;
//   rho' = (rt, r);  beta = (rho' / rho) (alpha / omega).
// The scalars live in device memory (BiState); each reduction is two-pass
// (per-block partials, then a one-block finish launch that updates the
// scalars), so the host only polls the state between batches of iterations.
// Every vector kernel of an iteration queued after the stop returns at once.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "device.h"
#include "internal.h"
#include "ops.h"

namespace tmqcd {
namespace {

struct BiK {
    int64_t stride, hbytes;
    int vh, nhalf;
};

__device__ __forceinline__ bool bi_site(const BiK& v, int i, int& half, int& h) {
    if (i >= v.nhalf * v.vh) return false;
    half = i / v.vh;
    h = i - half * v.vh;
    return true;
}

__device__ __forceinline__ C<double> cfrom(const double (&z)[2]) { return {z[0], z[1]}; }
__device__ __forceinline__ void cto(double (&z)[2], C<double> a) {
    z[0] = a.re;
    z[1] = a.im;
}
__device__ __forceinline__ C<double> cdivz(C<double> a, C<double> b) {
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

#define BI_LOAD(f, ptr) SpinorIO<TMQCD_F64>::load(f, (ptr) + half * v.hbytes, v.stride, h)
#define BI_STORE(ptr, f) SpinorIO<TMQCD_F64>::store((ptr) + half * v.hbytes, v.stride, h, f)

// p = r + beta (p - omega v)
__global__ __launch_bounds__(kBlock) void bi_p_kernel(BiK v, char* p, const char* r, const char* vv,
                                                      const BiState* st) {
    if (st->done) return;
    int half, h;
    if (!bi_site(v, blockIdx.x * kBlock + threadIdx.x, half, h)) return;
    const C<double> beta = cfrom(st->beta), omega = cfrom(st->omega);
    Spinor<double> pf, rf, vf;
    BI_LOAD(pf, p);
    BI_LOAD(rf, r);
    BI_LOAD(vf, vv);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) pf.s[s][c] = rf.s[s][c] + beta * (pf.s[s][c] - omega * vf.s[s][c]);
    BI_STORE(p, pf);
}

// partials of (a, b) = a^+ b (two doubles per block)
__global__ __launch_bounds__(kBlock) void bi_dot_kernel(BiK v, const char* a, const char* b, double* partials,
                                                        const BiState* st) {
    if (st->done) return;
    int half, h;
    double z[2] = {0.0, 0.0};
    if (bi_site(v, blockIdx.x * kBlock + threadIdx.x, half, h)) {
        Spinor<double> af, bf;
        BI_LOAD(af, a);
        BI_LOAD(bf, b);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const C<double> w = cmul_cj(af.s[s][c], bf.s[s][c]);
                z[0] += w.re;
                z[1] += w.im;
            }
    }
    block_partial<2>(z, partials, blockIdx.x);
}

// s = r - alpha v
__global__ __launch_bounds__(kBlock) void bi_s_kernel(BiK v, char* sv, const char* r, const char* vv,
                                                      const BiState* st) {
    if (st->done) return;
    int half, h;
    if (!bi_site(v, blockIdx.x * kBlock + threadIdx.x, half, h)) return;
    const C<double> alpha = cfrom(st->alpha);
    Spinor<double> rf, vf;
    BI_LOAD(rf, r);
    BI_LOAD(vf, vv);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) rf.s[s][c] = rf.s[s][c] - alpha * vf.s[s][c];
    BI_STORE(sv, rf);
}

// partials of (t, s) (complex) and (t, t)
__global__ __launch_bounds__(kBlock) void bi_ts_kernel(BiK v, const char* t, const char* sv, double* partials,
                                                       const BiState* st) {
    if (st->done) return;
    int half, h;
    double z[3] = {0.0, 0.0, 0.0};
    if (bi_site(v, blockIdx.x * kBlock + threadIdx.x, half, h)) {
        Spinor<double> tf, sf;
        BI_LOAD(tf, t);
        BI_LOAD(sf, sv);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const C<double> w = cmul_cj(tf.s[s][c], sf.s[s][c]);
                z[0] += w.re;
                z[1] += w.im;
                z[2] += norm2(tf.s[s][c]);
            }
    }
    block_partial<3>(z, partials, blockIdx.x);
}

// x += alpha p + omega s; r = s - omega t; partials of |r|^2 and (rt, r)
__global__ __launch_bounds__(kBlock) void bi_xr_kernel(BiK v, char* x, char* r, const char* p, const char* sv,
                                                       const char* t, const char* rt, double* partials,
                                                       const BiState* st) {
    if (st->done) return;
    int half, h;
    double z[3] = {0.0, 0.0, 0.0};
    if (bi_site(v, blockIdx.x * kBlock + threadIdx.x, half, h)) {
        const C<double> alpha = cfrom(st->alpha), omega = cfrom(st->omega);
        Spinor<double> xf, pf, sf, tf, rtf;
        BI_LOAD(xf, x);
        BI_LOAD(pf, p);
        BI_LOAD(sf, sv);
        BI_LOAD(tf, t);
        BI_LOAD(rtf, rt);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xf.s[s][c] = xf.s[s][c] + alpha * pf.s[s][c] + omega * sf.s[s][c];
                sf.s[s][c] = sf.s[s][c] - omega * tf.s[s][c];
                z[0] += norm2(sf.s[s][c]);
                const C<double> w = cmul_cj(rtf.s[s][c], sf.s[s][c]);
                z[1] += w.re;
                z[2] += w.im;
            }
        BI_STORE(x, xf);
        BI_STORE(r, sf);
    }
    block_partial<3>(z, partials, blockIdx.x);
}

// rt = r, p = 0, v = 0 at a (re)start
__global__ __launch_bounds__(kBlock) void bi_start_kernel(BiK v, char* rt, char* p, char* vv, const char* r) {
    int half, h;
    if (!bi_site(v, blockIdx.x * kBlock + threadIdx.x, half, h)) return;
    Spinor<double> rf, zf;
    BI_LOAD(rf, r);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) zf.s[s][c] = {0.0, 0.0};
    BI_STORE(rt, rf);
    BI_STORE(p, zf);
    BI_STORE(vv, zf);
}

#undef BI_LOAD
#undef BI_STORE

enum BiFinish { kBiAlpha = 0, kBiOmega = 1, kBiRho = 2 };

__device__ __forceinline__ bool cfinite(C<double> a) { return isfinite(a.re) && isfinite(a.im); }

// second pass of the three reductions and the scalar updates (one block)
template <int KIND>
__device__ __forceinline__ void bi_finish(BiState* st, const double* partials, int n) {
    constexpr int N = KIND == kBiAlpha ? 2 : 3;
    double tot[N];
    sum_partials<N>(partials, n, tot);
    if (threadIdx.x != 0) return;
    if constexpr (KIND == kBiAlpha) {
        const C<double> rv = {tot[0], tot[1]};
        const C<double> alpha = cdivz(cfrom(st->rho), rv);
        if (!(rv.re != 0.0 || rv.im != 0.0) || !cfinite(alpha)) {
            st->done = kDoneBreakdown;
            return;
        }
        cto(st->alpha, alpha);
    } else if constexpr (KIND == kBiOmega) {
        const double tt = tot[2];
        C<double> omega = {0.0, 0.0};
        if (tt > 0.0) omega = {tot[0] / tt, tot[1] / tt};
        if (!cfinite(omega)) {
            st->done = kDoneBreakdown;
            return;
        }
        cto(st->omega, omega);
    } else {
        const double rr = tot[0];
        const C<double> rho = {tot[1], tot[2]};
        st->rr = rr;
        st->iter += 1;
        if (!isfinite(rr)) {
            st->done = kDoneBreakdown;
        } else if (rr <= st->stop_rr) {
            st->done = kDoneStop;
        } else if (st->iter >= st->max_iter) {
            st->done = kDoneMaxIter;
        } else {
            const C<double> omega = cfrom(st->omega);
            if (!(omega.re != 0.0 || omega.im != 0.0) || !(rho.re != 0.0 || rho.im != 0.0)) {
                st->done = kDoneBreakdown;
                return;
            }
            const C<double> beta = cdivz(rho, cfrom(st->rho)) * cdivz(cfrom(st->alpha), omega);
            cto(st->beta, beta);
            cto(st->rho, rho);
        }
    }
}

__global__ __launch_bounds__(kBlock) void bi_finish_kernel(BiState* st, const double* partials, int n, int kind) {
    if (st->done) return;
    if (kind == kBiAlpha) bi_finish<kBiAlpha>(st, partials, n);
    else if (kind == kBiOmega) bi_finish<kBiOmega>(st, partials, n);
    else bi_finish<kBiRho>(st, partials, n);
}

// a (re)start: rho = (rt, r) = |r|^2 = rr, beta = rho (p = r in the first iteration), alpha = omega = 1
__global__ void bi_init_kernel(BiState* st, const CgState* cs, int slot, double stop_rr, int iter, int max_iter) {
    if (threadIdx.x != 0) return;
    const double rr = cs->result[slot];
    st->rr = rr;
    st->rho[0] = rr;
    st->rho[1] = 0.0;
    st->beta[0] = rr;
    st->beta[1] = 0.0;
    st->alpha[0] = st->omega[0] = 1.0;
    st->alpha[1] = st->omega[1] = 0.0;
    st->stop_rr = stop_rr;
    st->iter = iter;
    st->max_iter = max_iter;
    st->done = kDoneRunning;
}

BiK make_bik(const Geom& g, int nhalf) {
    BiK k;
    k.stride = g.stride;
    k.hbytes = half_field_bytes(g, TMQCD_F64);
    k.vh = (int)g.vh;
    k.nhalf = nhalf;
    return k;
}

struct BiFields {
    void *r, *rt, *p, *v, *s, *t, *ax, *tmp;
    BiState* st;
    CgState* cs;
    double* partials;
};

int64_t align_up(int64_t v) { return round_up(v, kAlignBytes); }

BiFields carve(const Geom& g, int op, char* base, int64_t* total) {
    const int64_t f = field_bytes(g, TMQCD_F64, op == TMQCD_M ? TMQCD_FULL : TMQCD_EVEN);
    const int nhalf = op == TMQCD_M ? 2 : 1;
    const int64_t nb = (nhalf * g.vh + kBlock - 1) / kBlock;
    int64_t off = 0;
    auto take = [&](int64_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    BiFields w;
    w.st = reinterpret_cast<BiState*>(take(sizeof(BiState)));
    w.cs = reinterpret_cast<CgState*>(take(sizeof(CgState)));
    // three values per block of the vector grid (the residual helpers use one per block of the same grid)
    w.partials = reinterpret_cast<double*>(take(8 * 3 * nb + 8 * kBlock));
    w.r = take(f);
    w.rt = take(f);
    w.p = take(f);
    w.v = take(f);
    w.s = take(f);
    w.t = take(f);
    w.ax = take(f);
    w.tmp = take(dslash_tmp_bytes(g, op, TMQCD_F64) + 1);
    if (total) *total = off;
    return w;
}

}  // namespace

int64_t bicgstab_workspace(const Geom& g, int op) {
    int64_t total = 0;
    carve(g, op, nullptr, &total);
    return total;
}

#define TRY(expr)                                     \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) {                       \
            g_last_hip_error = (int)e_;               \
            return TMQCD_EHIP;                        \
        }                                             \
    } while (0)

int run_bicgstab(const tmqcd_problem& prob, const void* gauge, const void* b, void* x, const tmqcd_cg_opts& o,
                 tmqcd_cg_stats& stats, void* ws, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    std::memset(&stats, 0, sizeof(stats));
    const Geom g = make_geom(prob);
    const int op = o.op;
    const int nhalf = op == TMQCD_M ? 2 : 1;
    const int hops_per_apply = op == TMQCD_M ? 1 : 2;
    BiFields w = carve(g, op, static_cast<char*>(ws), nullptr);
    const OpCtx c = make_ctx(prob, TMQCD_F64, o.recon, gauge, s);
    const VecSpec vs{&g, nhalf};
    const BiK k = make_bik(g, nhalf);
    const int nb = (int)((nhalf * g.vh + kBlock - 1) / kBlock);
    const dim3 grid(nb), block(kBlock);
    const int check = o.check_every > 0 ? o.check_every : 32;
    char* tmp = static_cast<char*>(w.tmp);

    int applies = 0;
    auto apply = [&](const void* in, void* out) -> hipError_t {
        ++applies;
        return apply_operator(c, op, in, out, tmp, 1);
    };
    auto read = [&](void* dst, const void* src, size_t n) -> hipError_t {
        hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s);
        return e == hipSuccess ? hipStreamSynchronize(s) : e;
    };
    // r = b - A x, |r|^2 -> cs->result[0]; |b|^2 -> cs->result[1]
    if (o.x_is_zero) {
        TRY(launch_zero(vs, x, TMQCD_F64, s));
        TRY(launch_convert(vs, w.r, TMQCD_F64, b, TMQCD_F64, s));
        TRY(launch_norm2(vs, w.r, TMQCD_F64, w.cs, 0, w.partials, s));
    } else {
        TRY(apply(x, w.ax));
        TRY(launch_residual(vs, w.r, b, w.ax, w.cs, 0, w.partials, s));
    }
    TRY(launch_norm2(vs, b, TMQCD_F64, w.cs, 1, w.partials, s));
    CgState hc;
    TRY(read(&hc, w.cs, sizeof(hc)));
    const double bb = hc.result[1];
    double rr = hc.result[0];
    if (!std::isfinite(rr) || !std::isfinite(bb)) return TMQCD_EBREAKDOWN;
    if (bb == 0.0) {
        TRY(launch_zero(vs, x, TMQCD_F64, s));
        stats.converged = 1;
        stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        TRY(hipStreamSynchronize(s));
        return TMQCD_OK;
    }
    const double target = o.tol * o.tol * bb;
    int iters = 0, status = TMQCD_OK;
    BiState hb;
    std::memset(&hb, 0, sizeof(hb));
    // restart from the true residual when the recursive one met the target but the true one did not
    constexpr int kMaxRestarts = 8;
    for (int restart = 0;; ++restart) {
        if (rr <= target) {
            stats.converged = 1;
            break;
        }
        if (restart > kMaxRestarts || iters >= o.max_iter) {
            status = TMQCD_ENOCONV;
            break;
        }
        hipLaunchKernelGGL(bi_start_kernel, grid, block, 0, s, k, static_cast<char*>(w.rt), static_cast<char*>(w.p),
                           static_cast<char*>(w.v), static_cast<const char*>(w.r));
        TRY(hipGetLastError());
        hipLaunchKernelGGL(bi_init_kernel, dim3(1), dim3(64), 0, s, w.st, static_cast<const CgState*>(w.cs), 0,
                           target, iters, o.max_iter);
        TRY(hipGetLastError());
        int batch = std::min(check, 8);
        for (;;) {
            for (int it = 0; it < batch; ++it) {
                hipLaunchKernelGGL(bi_p_kernel, grid, block, 0, s, k, static_cast<char*>(w.p),
                                   static_cast<const char*>(w.r), static_cast<const char*>(w.v), w.st);
                TRY(hipGetLastError());
                TRY(apply(w.p, w.v));
                hipLaunchKernelGGL(bi_dot_kernel, grid, block, 0, s, k, static_cast<const char*>(w.rt),
                                   static_cast<const char*>(w.v), w.partials, w.st);
                hipLaunchKernelGGL(bi_finish_kernel, dim3(1), block, 0, s, w.st, w.partials, nb, (int)kBiAlpha);
                hipLaunchKernelGGL(bi_s_kernel, grid, block, 0, s, k, static_cast<char*>(w.s),
                                   static_cast<const char*>(w.r), static_cast<const char*>(w.v), w.st);
                TRY(hipGetLastError());
                TRY(apply(w.s, w.t));
                hipLaunchKernelGGL(bi_ts_kernel, grid, block, 0, s, k, static_cast<const char*>(w.t),
                                   static_cast<const char*>(w.s), w.partials, w.st);
                hipLaunchKernelGGL(bi_finish_kernel, dim3(1), block, 0, s, w.st, w.partials, nb, (int)kBiOmega);
                hipLaunchKernelGGL(bi_xr_kernel, grid, block, 0, s, k, static_cast<char*>(x), static_cast<char*>(w.r),
                                   static_cast<const char*>(w.p), static_cast<const char*>(w.s),
                                   static_cast<const char*>(w.t), static_cast<const char*>(w.rt), w.partials, w.st);
                hipLaunchKernelGGL(bi_finish_kernel, dim3(1), block, 0, s, w.st, w.partials, nb, (int)kBiRho);
                TRY(hipGetLastError());
            }
            TRY(read(&hb, w.st, sizeof(hb)));
            if (hb.done != kDoneRunning) break;
            batch = check;
        }
        iters = hb.iter;
        // the true residual of x
        TRY(apply(x, w.ax));
        TRY(launch_residual(vs, w.r, b, w.ax, w.cs, 0, w.partials, s));
        TRY(read(&hc, w.cs, sizeof(hc)));
        rr = hc.result[0];
        stats.reliable_updates += 1;
        stats.iter_rel_residual = std::sqrt(hb.rr / bb);
        if (!std::isfinite(rr)) {
            status = TMQCD_EBREAKDOWN;
            break;
        }
        if (rr <= target) {
            stats.converged = 1;
            break;
        }
        if (hb.done == kDoneBreakdown) {
            status = TMQCD_EBREAKDOWN;
            break;
        }
        if (hb.done == kDoneMaxIter) {
            status = TMQCD_ENOCONV;
            break;
        }
    }
    // applications queued past the stop are counted too: they were launched
    stats.iters = iters;
    stats.hop_launches = hops_per_apply * applies;
    stats.true_rel_residual = std::sqrt(rr / bb);
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

}  // namespace tmqcd
