// BLAS-1 on packed spinor fields (the paper's "LAPACK" kernels: saxpy and
// scalar products) with deterministic FP64 reductions, plus the solver-state
// kernels that keep CG scalars on the device.
#include "device.h"
#include "internal.h"

namespace tmqcd {
namespace {

struct VecK {
    int64_t stride;
    int vh;
    int nhalf;
    int nblocks;
};

__device__ __forceinline__ bool site_of(const VecK& v, int i, int& half, int& h) {
    if (i >= v.nhalf * v.vh) return false;
    half = i / v.vh;
    h = i - half * v.vh;
    return true;
}

VecK make_veck(const VecSpec& s) {
    VecK k;
    k.stride = s.g->stride;
    k.vh = (int)s.g->vh;
    k.nhalf = s.nhalf;
    k.nblocks = (int)((s.nhalf * s.g->vh + kBlock - 1) / kBlock);
    return k;
}

template <int PD, int PS>
__global__ __launch_bounds__(kBlock) void convert_kernel(VecK v, char* dst, int64_t dbytes, const char* src,
                                                         int64_t sbytes) {
    int half, h;
    if (!site_of(v, blockIdx.x * kBlock + threadIdx.x, half, h)) return;
    Spinor<double> a;
    if constexpr (PS == TMQCD_F64) {
        SpinorIO<TMQCD_F64>::load(a, src + half * sbytes, v.stride, h);
    } else {
        Spinor<float> b;
        SpinorIO<PS>::load(b, src + half * sbytes, v.stride, h);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) a.s[s][c] = {(double)b.s[s][c].re, (double)b.s[s][c].im};
    }
    if constexpr (PD == TMQCD_F64) {
        SpinorIO<TMQCD_F64>::store(dst + half * dbytes, v.stride, h, a);
    } else {
        Spinor<float> b;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) b.s[s][c] = {(float)a.s[s][c].re, (float)a.s[s][c].im};
        SpinorIO<PD>::store(dst + half * dbytes, v.stride, h, b);
    }
}

template <int P>
__global__ __launch_bounds__(kBlock) void norm2_kernel(VecK v, const char* src, int64_t bytes, double* partials) {
    int half, h;
    double red = 0;
    if (site_of(v, blockIdx.x * kBlock + threadIdx.x, half, h)) {
        Spinor<typename Prec<P>::T> a;
        SpinorIO<P>::load(a, src + half * bytes, v.stride, h);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) red += (double)norm2(a.s[s][c]);
    }
    const double in[1] = {red};
    block_partial<1>(in, partials, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void residual_kernel(VecK v, char* r, const char* b, const char* ax,
                                                          int64_t bytes, double* partials) {
    int half, h;
    double red = 0;
    if (site_of(v, blockIdx.x * kBlock + threadIdx.x, half, h)) {
        Spinor<double> bv, av;
        SpinorIO<TMQCD_F64>::load(bv, b + half * bytes, v.stride, h);
        SpinorIO<TMQCD_F64>::load(av, ax + half * bytes, v.stride, h);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                bv.s[s][c] = bv.s[s][c] - av.s[s][c];
                red += norm2(bv.s[s][c]);
            }
        SpinorIO<TMQCD_F64>::store(r + half * bytes, v.stride, h, bv);
    }
    const double in[1] = {red};
    block_partial<1>(in, partials, blockIdx.x);
}

template <int PP, int PR>
__global__ __launch_bounds__(kBlock) void xpay_kernel(VecK v, char* p, int64_t pbytes, const char* r, int64_t rbytes,
                                                      const CgState* st, int skip_if_done) {
    if (skip_if_done && st->done) return;
    int half, h;
    if (!site_of(v, blockIdx.x * kBlock + threadIdx.x, half, h)) return;
    using T = typename Prec<PP>::T;
    const T beta = (T)st->beta;
    Spinor<T> pv, rv;
    SpinorIO<PP>::load(pv, p + half * pbytes, v.stride, h);
    SpinorIO<PR>::load(rv, r + half * rbytes, v.stride, h);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) pv.s[s][c] = rv.s[s][c] + scale(beta, pv.s[s][c]);
    SpinorIO<PP>::store(p + half * pbytes, v.stride, h, pv);
}

// x += alpha p and p = r + beta p inside the CG iteration: beta = rr_new / rr with
// rr_new the sum of the update hop's partials, formed by every block in the same fixed
// order (so all blocks use the same beta) while st->rr still holds the previous |r|^2;
// the state itself is updated by the next launch that finishes the pending beta.
// x (precision PR, as r) is updated here from the p this launch reads anyway, not in
// the update hop.
template <int PP, int PR>
__global__ __launch_bounds__(kBlock) void xpay_fused_kernel(VecK v, char* p, int64_t pbytes, const char* r,
                                                            int64_t rbytes, char* x, CgState* st,
                                                            const double* partials, int n) {
    if (block_stopped(st)) return;
    double tot[1];
    sum_partials<1>(partials, n, tot);
    const double beta_d = tot[0] / st->rr;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->beta_pending = 1;
    // The pending finish will stop the recursion here (the stop tests of
    // cg_finish_update, on the same total): x takes this iteration's step, and p keeps
    // the last search direction, from which a reliable update restarts, as when the
    // finish precedes p.
    const int it = st->iter + 1;
    const bool stops = !isfinite(tot[0]) || tot[0] <= st->stop_rr || it >= st->cycle_end || it >= st->max_iter;
    int half, h;
    if (!site_of(v, blockIdx.x * kBlock + threadIdx.x, half, h)) return;
    using T = typename Prec<PP>::T;
    const T alpha = (T)st->alpha, beta = (T)beta_d;
    Spinor<T> pv, xv;
    SpinorIO<PP>::load(pv, p + half * pbytes, v.stride, h);
    SpinorIO<PR>::load(xv, x + half * rbytes, v.stride, h);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) xv.s[s][c] = xv.s[s][c] + scale(alpha, pv.s[s][c]);
    SpinorIO<PR>::store(x + half * rbytes, v.stride, h, xv);
    if (stops) return;
    Spinor<T> rv;
    SpinorIO<PR>::load(rv, r + half * rbytes, v.stride, h);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) pv.s[s][c] = rv.s[s][c] + scale(beta, pv.s[s][c]);
    SpinorIO<PP>::store(p + half * pbytes, v.stride, h, pv);
}

constexpr int kMaxBatchVec = 8;
struct XpayBatch {
    int n;
    int tile_start[kMaxBatchVec + 1];
    VecK v[kMaxBatchVec];
    char* p[kMaxBatchVec];
    const char* r[kMaxBatchVec];
    char* x[kMaxBatchVec];
    CgState* st[kMaxBatchVec];
    const double* partials[kMaxBatchVec];   // the update hop's |r|^2 partials of each lattice
    int np[kMaxBatchVec];
    int64_t bytes;
};

// The batched CG's search-direction update, as xpay_fused_kernel for several lattices
// (FP64), grid-stride over their tiles: every tile forms its lattice's beta from the
// update hop's partials, x += alpha p, and p = r + beta p unless the pending finish will
// stop the lattice at this iteration; the lattice's first tile marks that finish
// pending (the next iteration's first hop, or the finish before the host reads, does it).
__global__ __launch_bounds__(kBlock) void xpay_batch_kernel(const XpayBatch b) {
    const int total = b.tile_start[b.n];
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        int i = 0;
        while (tile >= b.tile_start[i + 1]) ++i;
        CgState* st = b.st[i];
        if (block_stopped(st)) continue;   // block-uniform
        double tot[1];
        sum_partials<1>(b.partials[i], b.np[i], tot);
        const double beta = tot[0] / st->rr;
        if (tile == b.tile_start[i] && threadIdx.x == 0) st->beta_pending = 1;
        const int it = st->iter + 1;
        const bool stops = !isfinite(tot[0]) || tot[0] <= st->stop_rr || it >= st->cycle_end || it >= st->max_iter;
        int half, h;
        if (!site_of(b.v[i], (tile - b.tile_start[i]) * kBlock + threadIdx.x, half, h)) continue;
        const double alpha = st->alpha;
        Spinor<double> pv, xv;
        SpinorIO<TMQCD_F64>::load(pv, b.p[i] + half * b.bytes, b.v[i].stride, h);
        SpinorIO<TMQCD_F64>::load(xv, b.x[i] + half * b.bytes, b.v[i].stride, h);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) xv.s[s][c] = xv.s[s][c] + scale(alpha, pv.s[s][c]);
        SpinorIO<TMQCD_F64>::store(b.x[i] + half * b.bytes, b.v[i].stride, h, xv);
        if (stops) continue;
        Spinor<double> rv;
        SpinorIO<TMQCD_F64>::load(rv, b.r[i] + half * b.bytes, b.v[i].stride, h);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) pv.s[s][c] = rv.s[s][c] + scale(beta, pv.s[s][c]);
        SpinorIO<TMQCD_F64>::store(b.p[i] + half * b.bytes, b.v[i].stride, h, pv);
    }
}

template <int PS>
__global__ __launch_bounds__(kBlock) void accumulate_kernel(VecK v, char* x, int64_t xbytes, char* xs,
                                                            int64_t sbytes) {
    int half, h;
    if (!site_of(v, blockIdx.x * kBlock + threadIdx.x, half, h)) return;
    Spinor<double> a;
    Spinor<float> b;
    SpinorIO<TMQCD_F64>::load(a, x + half * xbytes, v.stride, h);
    SpinorIO<PS>::load(b, xs + half * sbytes, v.stride, h);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a.s[s][c] = {a.s[s][c].re + (double)b.s[s][c].re, a.s[s][c].im + (double)b.s[s][c].im};
            b.s[s][c] = {0.f, 0.f};
        }
    SpinorIO<TMQCD_F64>::store(x + half * xbytes, v.stride, h, a);
    SpinorIO<PS>::store(xs + half * sbytes, v.stride, h, b);
}

template <int P>
__global__ __launch_bounds__(kBlock) void zero_kernel(VecK v, char* dst, int64_t bytes) {
    int half, h;
    if (!site_of(v, blockIdx.x * kBlock + threadIdx.x, half, h)) return;
    Spinor<typename Prec<P>::T> a;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) a.s[s][c] = {0, 0};
    SpinorIO<P>::store(dst + half * bytes, v.stride, h, a);
}

// deterministic, site-dependent test values in [-1, 1) (for tuning runs)
template <int P>
__global__ __launch_bounds__(kBlock) void fill_kernel(VecK v, char* dst, int64_t bytes, unsigned seed) {
    int half, h;
    if (!site_of(v, blockIdx.x * kBlock + threadIdx.x, half, h)) return;
    Spinor<typename Prec<P>::T> a;
    unsigned x = (unsigned)(half * v.vh + h) * 2654435761u ^ seed;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x = x * 1664525u + 1013904223u;
            const float re = (float)(x >> 8) * (1.0f / 8388608.0f) - 1.0f;
            x = x * 1664525u + 1013904223u;
            const float im = (float)(x >> 8) * (1.0f / 8388608.0f) - 1.0f;
            a.s[s][c] = {re, im};
        }
    SpinorIO<P>::store(dst + half * bytes, v.stride, h, a);
}

// number of 8-byte words that differ between two buffers
__global__ __launch_bounds__(kBlock) void compare_kernel(const unsigned long long* a, const unsigned long long* b,
                                                         int64_t n, unsigned long long* mismatches) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        c += a[i] != b[i];
    if (c) atomicAdd(mismatches, c);
}

__global__ void set_state_kernel(CgState* st, StateInit v) {
    if (threadIdx.x != 0) return;
    if (v.set_rr) st->rr = v.rr;
    if (v.set_rr_prev) st->rr_prev = v.rr_prev;
    if (v.set_stop) st->stop_rr = v.stop_rr;
    if (v.set_alpha) st->alpha = v.alpha;
    if (v.set_beta) st->beta = v.beta;
    if (v.set_iter) st->iter = v.iter;
    if (v.set_max_iter) st->max_iter = v.max_iter;
    if (v.set_cycle_end) st->cycle_end = v.cycle_end;
    if (v.set_done) {   // a solve (re)starts or stops here: no beta finish or x update is pending
        st->done = v.done;
        st->beta_pending = 0;
        st->x_pending = 0;
    }
}

__global__ void rr_from_result_kernel(CgState* st, int slot, double stop_factor) {
    if (threadIdx.x != 0) return;
    const double rr = st->result[slot];
    st->rr = rr;
    if (stop_factor > 0) st->stop_rr = stop_factor * rr;
}

// second pass of a standalone reduction: st->result[slot] = sum of the partials
__global__ __launch_bounds__(kBlock) void result_finish_kernel(CgState* st, const double* partials, int n, int slot) {
    double tot[1];
    sum_partials<1>(partials, n, tot);
    if (threadIdx.x == 0) st->result[slot] = tot[0];
}

// second pass of the CG reductions; block b serves lattice b
constexpr int kMaxFinish = 8;
struct FinishBatch {
    CgState* st[kMaxFinish];
    const double* partials[kMaxFinish];
    int n[kMaxFinish];
};

static_assert(kFinishAlpha == 0 && kFinishBeta == 1 && kFinishBetaPending == 2,
              "finish kinds as cg_finish_block numbers them");

__global__ __launch_bounds__(kBlock) void cg_finish_kernel(const FinishBatch f, int kind) {
    cg_finish_block<kBlock>(f.st[blockIdx.x], f.partials[blockIdx.x], f.n[blockIdx.x], kind);
}

// The multi-RHS CG: block b finishes column b's reduction (tiles partials at partials + b * tiles).
__global__ __launch_bounds__(kBlock) void cg_finish_cols_kernel(CgState* st, const double* partials, int tiles,
                                                                int kind) {
    cg_finish_block<kBlock>(st + blockIdx.x, partials + (int64_t)blockIdx.x * tiles, tiles, kind);
}

// p_c = r_c + beta_c p_c for every column c = blockIdx.y whose solve runs (FP64 fields fstride apart).
__global__ __launch_bounds__(kBlock) void xpay_cols_kernel(VecK v, char* p, const char* r, char* x, int64_t hbytes,
                                                           int64_t fstride, const CgState* st) {
    const int c = blockIdx.y;
    // x += alpha p for a column whose r update ran in this iteration (also the one that stopped
    // it), then p = r + beta p while the column runs
    const bool upd_x = st[c].x_pending != 0, upd_p = st[c].done == 0;
    if (!upd_x && !upd_p) return;
    int half, h;
    if (!site_of(v, blockIdx.x * kBlock + threadIdx.x, half, h)) return;
    char* pc = p + c * fstride + half * hbytes;
    Spinor<double> pv;
    SpinorIO<TMQCD_F64>::load(pv, pc, v.stride, h);
    if (upd_x) {
        const double alpha = st[c].alpha;
        char* xc = x + c * fstride + half * hbytes;
        Spinor<double> xv;
        SpinorIO<TMQCD_F64>::load(xv, xc, v.stride, h);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 3; ++k) xv.s[s][k] = xv.s[s][k] + scale(alpha, pv.s[s][k]);
        SpinorIO<TMQCD_F64>::store(xc, v.stride, h, xv);
    }
    if (!upd_p) return;
    const double beta = st[c].beta;
    Spinor<double> rv;
    SpinorIO<TMQCD_F64>::load(rv, r + c * fstride + half * hbytes, v.stride, h);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k) pv.s[s][k] = rv.s[s][k] + scale(beta, pv.s[s][k]);
    SpinorIO<TMQCD_F64>::store(pc, v.stride, h, pv);
}

template <template <int> class F, typename... A>
hipError_t by_prec(int p, A... a) {
    switch (p) {
        case TMQCD_F64: return F<TMQCD_F64>::run(a...);
        case TMQCD_F32: return F<TMQCD_F32>::run(a...);
        case TMQCD_F16: return F<TMQCD_F16>::run(a...);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_convert(const VecSpec& v, void* dst, int pdst, const void* src, int psrc, hipStream_t s) {
    const VecK k = make_veck(v);
    char* d = static_cast<char*>(dst);
    const char* sr = static_cast<const char*>(src);
    const int64_t db = half_field_bytes(*v.g, pdst), sb = half_field_bytes(*v.g, psrc);
#define TMQCD_CONV(A, B)                                                                                       \
    if (pdst == A && psrc == B) {                                                                              \
        hipLaunchKernelGGL((convert_kernel<A, B>), dim3(k.nblocks), dim3(kBlock), 0, s, k, d, db, sr, sb);    \
        return hipGetLastError();                                                                              \
    }
    TMQCD_CONV(TMQCD_F64, TMQCD_F64)
    TMQCD_CONV(TMQCD_F32, TMQCD_F64)
    TMQCD_CONV(TMQCD_F16, TMQCD_F64)
    TMQCD_CONV(TMQCD_F64, TMQCD_F32)
    TMQCD_CONV(TMQCD_F64, TMQCD_F16)
    TMQCD_CONV(TMQCD_F32, TMQCD_F32)
    TMQCD_CONV(TMQCD_F16, TMQCD_F32)
    TMQCD_CONV(TMQCD_F32, TMQCD_F16)
    TMQCD_CONV(TMQCD_F16, TMQCD_F16)
#undef TMQCD_CONV
    return hipErrorInvalidValue;
}

namespace {
template <int P>
struct Norm2Run {
    static hipError_t run(const VecK k, const char* src, int64_t bytes, double* partials, hipStream_t s) {
        hipLaunchKernelGGL((norm2_kernel<P>), dim3(k.nblocks), dim3(kBlock), 0, s, k, src, bytes, partials);
        return hipGetLastError();
    }
};
hipError_t result_finish(CgState* st, const double* partials, int n, int slot, hipStream_t s) {
    hipLaunchKernelGGL(result_finish_kernel, dim3(1), dim3(kBlock), 0, s, st, partials, n, slot);
    return hipGetLastError();
}
template <int P>
struct ZeroRun {
    static hipError_t run(const VecK k, char* dst, int64_t bytes, hipStream_t s) {
        hipLaunchKernelGGL((zero_kernel<P>), dim3(k.nblocks), dim3(kBlock), 0, s, k, dst, bytes);
        return hipGetLastError();
    }
};
}  // namespace

hipError_t launch_norm2(const VecSpec& v, const void* src, int prec, CgState* st, int slot, double* partials,
                        hipStream_t s) {
    const VecK k = make_veck(v);
    const hipError_t e =
        by_prec<Norm2Run>(prec, k, static_cast<const char*>(src), half_field_bytes(*v.g, prec), partials, s);
    return e == hipSuccess ? result_finish(st, partials, k.nblocks, slot, s) : e;
}

hipError_t launch_zero(const VecSpec& v, void* dst, int prec, hipStream_t s) {
    return by_prec<ZeroRun>(prec, make_veck(v), static_cast<char*>(dst), half_field_bytes(*v.g, prec), s);
}

hipError_t launch_residual(const VecSpec& v, void* r, const void* b, const void* ax, CgState* st, int slot,
                           double* partials, hipStream_t s) {
    const VecK k = make_veck(v);
    hipLaunchKernelGGL(residual_kernel, dim3(k.nblocks), dim3(kBlock), 0, s, k, static_cast<char*>(r),
                       static_cast<const char*>(b), static_cast<const char*>(ax), half_field_bytes(*v.g, TMQCD_F64),
                       partials);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? result_finish(st, partials, k.nblocks, slot, s) : e;
}

hipError_t launch_xpay(const VecSpec& v, void* p, int pp, const void* r, int pr, CgState* st, bool skip_if_done,
                       hipStream_t s) {
    const VecK k = make_veck(v);
    char* pc = static_cast<char*>(p);
    const char* rc = static_cast<const char*>(r);
    const int64_t pb = half_field_bytes(*v.g, pp), rb = half_field_bytes(*v.g, pr);
    const int skip = skip_if_done ? 1 : 0;
    if (pp == TMQCD_F64 && pr == TMQCD_F64)
        hipLaunchKernelGGL((xpay_kernel<TMQCD_F64, TMQCD_F64>), dim3(k.nblocks), dim3(kBlock), 0, s, k, pc, pb, rc, rb, st, skip);
    else if (pp == TMQCD_F32 && pr == TMQCD_F32)
        hipLaunchKernelGGL((xpay_kernel<TMQCD_F32, TMQCD_F32>), dim3(k.nblocks), dim3(kBlock), 0, s, k, pc, pb, rc, rb, st, skip);
    else if (pp == TMQCD_F16 && pr == TMQCD_F32)
        hipLaunchKernelGGL((xpay_kernel<TMQCD_F16, TMQCD_F32>), dim3(k.nblocks), dim3(kBlock), 0, s, k, pc, pb, rc, rb, st, skip);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_xpay_fused(const VecSpec& v, void* p, int pp, const void* r, int pr, void* x, CgState* st,
                             const double* partials, int n, hipStream_t s) {
    const VecK k = make_veck(v);
    char* pc = static_cast<char*>(p);
    const char* rc = static_cast<const char*>(r);
    char* xc = static_cast<char*>(x);
    const int64_t pb = half_field_bytes(*v.g, pp), rb = half_field_bytes(*v.g, pr);
    if (pp == TMQCD_F64 && pr == TMQCD_F64)
        hipLaunchKernelGGL((xpay_fused_kernel<TMQCD_F64, TMQCD_F64>), dim3(k.nblocks), dim3(kBlock), 0, s, k, pc, pb,
                           rc, rb, xc, st, partials, n);
    else if (pp == TMQCD_F32 && pr == TMQCD_F32)
        hipLaunchKernelGGL((xpay_fused_kernel<TMQCD_F32, TMQCD_F32>), dim3(k.nblocks), dim3(kBlock), 0, s, k, pc, pb,
                           rc, rb, xc, st, partials, n);
    else if (pp == TMQCD_F16 && pr == TMQCD_F32)
        hipLaunchKernelGGL((xpay_fused_kernel<TMQCD_F16, TMQCD_F32>), dim3(k.nblocks), dim3(kBlock), 0, s, k, pc, pb,
                           rc, rb, xc, st, partials, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_accumulate(const VecSpec& v, void* x64, void* xs, int ps, hipStream_t s) {
    const VecK k = make_veck(v);
    const int64_t xb = half_field_bytes(*v.g, TMQCD_F64), sb = half_field_bytes(*v.g, ps);
    if (ps == TMQCD_F32)
        hipLaunchKernelGGL((accumulate_kernel<TMQCD_F32>), dim3(k.nblocks), dim3(kBlock), 0, s, k,
                           static_cast<char*>(x64), xb, static_cast<char*>(xs), sb);
    else if (ps == TMQCD_F16)
        hipLaunchKernelGGL((accumulate_kernel<TMQCD_F16>), dim3(k.nblocks), dim3(kBlock), 0, s, k,
                           static_cast<char*>(x64), xb, static_cast<char*>(xs), sb);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_set_state(CgState* st, const StateInit& v, hipStream_t s) {
    hipLaunchKernelGGL(set_state_kernel, dim3(1), dim3(64), 0, s, st, v);
    return hipGetLastError();
}

hipError_t launch_cg_finish_batch(CgState* const* st, const double* const* partials, const int* n, int count,
                                  int kind, hipStream_t s) {
    if (count < 1 || count > kMaxFinish) return hipErrorInvalidValue;
    FinishBatch f;
    for (int i = 0; i < count; ++i) {
        f.st[i] = st[i];
        f.partials[i] = partials[i];
        f.n[i] = n[i];
    }
    hipLaunchKernelGGL(cg_finish_kernel, dim3(count), dim3(kBlock), 0, s, f, kind);
    return hipGetLastError();
}

hipError_t launch_cg_finish(CgState* st, const double* partials, int n, int kind, hipStream_t s) {
    return launch_cg_finish_batch(&st, &partials, &n, 1, kind, s);
}

hipError_t launch_cg_finish_cols(CgState* st, const double* partials, int tiles, int ncol, int kind, hipStream_t s) {
    if (ncol < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cg_finish_cols_kernel, dim3(ncol), dim3(kBlock), 0, s, st, partials, tiles, kind);
    return hipGetLastError();
}

hipError_t launch_xpay_cols(const VecSpec& v, void* p, const void* r, void* x, int64_t fstride, int ncol,
                            const CgState* st, hipStream_t s) {
    const VecK k = make_veck(v);
    if (ncol < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(xpay_cols_kernel, dim3(k.nblocks, ncol), dim3(kBlock), 0, s, k, static_cast<char*>(p),
                       static_cast<const char*>(r), static_cast<char*>(x), half_field_bytes(*v.g, TMQCD_F64), fstride,
                       st);
    return hipGetLastError();
}

hipError_t launch_rr_from_result(CgState* st, int slot, double stop_factor, hipStream_t s) {
    hipLaunchKernelGGL(rr_from_result_kernel, dim3(1), dim3(64), 0, s, st, slot, stop_factor);
    return hipGetLastError();
}

hipError_t launch_xpay_batch(const VecSpec* vs, void* const* p, const void* const* r, void* const* x,
                             CgState* const* st, const double* const* partials, const int* np, int n, int max_grid,
                             hipStream_t s) {
    if (n < 1 || n > kMaxBatchVec) return hipErrorInvalidValue;
    XpayBatch b;
    b.n = n;
    b.tile_start[0] = 0;
    b.bytes = half_field_bytes(*vs[0].g, TMQCD_F64);
    for (int i = 0; i < n; ++i) {
        b.v[i] = make_veck(vs[i]);
        b.p[i] = static_cast<char*>(p[i]);
        b.r[i] = static_cast<const char*>(r[i]);
        b.x[i] = static_cast<char*>(x[i]);
        b.st[i] = st[i];
        b.partials[i] = partials[i];
        b.np[i] = np[i];
        b.tile_start[i + 1] = b.tile_start[i] + b.v[i].nblocks;
    }
    for (int i = 0; i < n; ++i)
        if (vs[i].nhalf != 1) return hipErrorInvalidValue;   // even-site fields only
    const int total = b.tile_start[n];
    hipLaunchKernelGGL(xpay_batch_kernel, dim3(total < max_grid ? total : max_grid), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

namespace {
template <int P>
struct FillRun {
    static hipError_t run(const VecK k, char* dst, int64_t bytes, unsigned seed, hipStream_t s) {
        hipLaunchKernelGGL((fill_kernel<P>), dim3(k.nblocks), dim3(kBlock), 0, s, k, dst, bytes, seed);
        return hipGetLastError();
    }
};
}  // namespace

hipError_t launch_fill(const VecSpec& v, void* dst, int prec, unsigned seed, hipStream_t s) {
    return by_prec<FillRun>(prec, make_veck(v), static_cast<char*>(dst), half_field_bytes(*v.g, prec), seed, s);
}

hipError_t launch_compare(const void* a, const void* b, int64_t bytes, unsigned long long* mismatches, hipStream_t s) {
    const int64_t n = bytes / 8;
    hipLaunchKernelGGL(compare_kernel, dim3(1024), dim3(kBlock), 0, s, static_cast<const unsigned long long*>(a),
                       static_cast<const unsigned long long*>(b), n, mismatches);
    return hipGetLastError();
}

}  // namespace tmqcd
