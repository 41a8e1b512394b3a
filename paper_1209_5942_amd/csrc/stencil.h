// The even-odd hop stencil shared by the single-RHS, multi-RHS and batched
// kernels (paper, section 2.1: the hopping part of D_tm; the storage-format
// section for the parity-split SoA layout).
//
// One thread per output site.  For each of the 8 directions the neighbour
// spinor is spin-projected to a half spinor with (1 -+ gamma_mu), multiplied by
// U_mu(x) or U_mu(x - mu)^+, and the lower spin components are rebuilt from the
// upper ones (the projectors have rank 2), which gives the standard 1320 flops
// per site.  The epilogue applies the twisted diagonal and, inside CG, the
// solver update and a deterministic FP64 reduction.
#pragma once

#include "device.h"
#include "internal.h"

namespace tmqcd {
namespace stencil {

// gamma_mu = [[0, B], [B^+, 0]] in the chiral basis.  Row r of B has its one
// nonzero in column kPerm[mu][r], equal to i^kB[mu][r]; row r of B^+ has it in
// the same column, equal to i^kBd[mu][r].
constexpr int kPerm[4][2] = {{1, 0}, {1, 0}, {0, 1}, {0, 1}};
constexpr int kB[4][2] = {{3, 3}, {2, 0}, {3, 1}, {2, 2}};
constexpr int kBd[4][2] = {{1, 1}, {0, 2}, {1, 3}, {2, 2}};

// (1 + eps gamma_mu) psi = [h ; eps B^+ h] with h = psi_up + eps B psi_dn
template <int MU, int EPS, int R, typename T>
__device__ __forceinline__ void project_row(Half<T>& h, const Spinor<T>& v) {
    constexpr int code = kB[MU][R] + (EPS > 0 ? 0 : 2);
    constexpr int src = 2 + kPerm[MU][R];
#pragma unroll
    for (int c = 0; c < 3; ++c) h.s[R][c] = v.s[R][c] + mul_i<code>(v.s[src][c]);
}
template <int MU, int EPS, int R, typename T>
__device__ __forceinline__ void accumulate_row(Spinor<T>& acc, const Half<T>& g) {
    constexpr int code = kBd[MU][R] + (EPS > 0 ? 0 : 2);
    constexpr int src = kPerm[MU][R];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc.s[R][c] = acc.s[R][c] + g.s[R][c];
        acc.s[2 + R][c] = acc.s[2 + R][c] + mul_i<code>(g.s[src][c]);
    }
}

template <bool ADJ, typename T>
__device__ __forceinline__ void su3_mul(Half<T>& g, const Su3<T>& u, const Half<T>& h) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if constexpr (ADJ) {
                g.s[r][a] = cmul_cj(u.m[0][a], h.s[r][0]) + cmul_cj(u.m[1][a], h.s[r][1]) + cmul_cj(u.m[2][a], h.s[r][2]);
            } else {
                g.s[r][a] = u.m[a][0] * h.s[r][0] + u.m[a][1] * h.s[r][1] + u.m[a][2] * h.s[r][2];
            }
        }
}

struct HopK {
    const char* gauge;
    const char* in;
    const char* own;
    char* out;
    char* r;                 // CG update: the residual, r -= alpha (A p)
    CgState* st;
    double* partials;
    int64_t stride, gstride, hbytes, vhbytes;
    int L[4];
    int lxh, vh, nb_half, nblocks, out_parity, nparity;
    int order, width;        // block order (kOrder*) and output sites per block
    int slice, q, tq, lt;    // slab orders: half sites per t-slice, per z-range, blocks per (slice, range)
    int nz, tlen;            // slab orders: z-ranges per slice, slices per t-range
    int by, bz, nry, nreg;   // column order: region extent in y and z, regions in y, regions
    const double* fin_partials;   // the previous launch's reduction, finished by block 0 first
    int fin_n, fin_kind;
    C<double> bc[4];
    C<double> cu_own, cd_own, cu_hop, cd_hop;
};

// The output site of lane `lane` of block b: parity and half index; false
// if the lane has no site.  The orders (which sites a block covers):
//  kOrderLinear:   block b covers half sites [b w, b w + w) of its parity;
//  kOrderXcdRemap: the same after the per-XCD remap of the block index (each
//                  XCD gets a contiguous range of tiles);
//  kOrderSlab:     the half sites of every t-slice are cut into 8 contiguous
//                  ranges of q sites (runs of z-planes), range x belonging to
//                  XCD x (hardware blocks go round-robin over the XCDs); each
//                  XCD walks through its ranges slice by slice, so the
//                  t-neighbours it reads belong to slices it has in flight;
//  kOrderSlabT2/4: the same with the lattice cut into nz = 4 (2) z-ranges
//                  times nt = 2 (4) t-ranges, XCD x owning z-range x % nz of
//                  t-range x / nz: half (a quarter) of the faces between the
//                  XCDs' z-ranges, for one t-face per t-range and a working
//                  set per slice twice (four times) as large;
//  kOrderColumn:   the (y, z) plane is cut into regions of by x bz (all x), and
//                  XCD x sweeps its regions x, x + 8, ... one after the other,
//                  each through all t: the neighbours an XCD reads lie in the
//                  few slices of one column it has in flight, except on the
//                  region's y and z faces.
__device__ __forceinline__ bool block_site(const HopK& a, int b, int lane, int& par, int& h) {
    if (a.order == kOrderXcdRemap) b = xcd_swizzle(b, a.nblocks);
    int lb = b;
    par = a.out_parity;
    if (a.nparity == 2) {
        par = b >= a.nb_half ? 1 : 0;
        lb = b - par * a.nb_half;
    }
    if (a.order == kOrderLinear || a.order == kOrderXcdRemap) {
        h = lb * a.width + lane;
        return h < a.vh;
    }
    const int x = lb & (kNumXcd - 1), k = lb / kNumXcd;
    if (slab_order(a.order)) {
        const int zr = x % a.nz, tr = x / a.nz;
        const int tl = k / a.tq, j = k - tl * a.tq;
        const int t = tr * a.tlen + tl;
        const int first = zr * a.q + j * a.width + lane;
        const int end = min((zr + 1) * a.q, a.slice);
        h = t * a.slice + first;
        return t < a.lt && first < end;
    }
    const int per = a.lt * a.tq;             // blocks per region
    const int ri = k / per, rem = k - ri * per;
    const int t = rem / a.tq, j = rem - t * a.tq;
    const int r = ri * kNumXcd + x;
    const int idx = j * a.width + lane;
    const int xh = idx % a.lxh, rest = idx / a.lxh;
    const int y = (r % a.nry) * a.by + rest % a.by;
    const int z = (r / a.nry) * a.bz + rest / a.by;
    h = xh + a.lxh * (y + a.L[1] * (z + a.L[2] * t));
    return r < a.nreg && rest < a.by * a.bz && y < a.L[1] && z < a.L[2];
}

// One of the eight terms: FWD: b+ (1 -+ gamma_mu) U_mu(x) psi(x+mu);
// backward: b- (1 +- gamma_mu) U_mu(x-mu)^+ psi(x-mu) (signs flip for H^+).
// The link is read from `lbase` in the packed link layout with stride
// `lstride` (global memory, or a block's link tile in LDS).  A hop across the
// boundary (`cross`) takes the boundary phase.  BRANCHLESS selects the factor
// (1 or the phase) and always multiplies: the term is then branch-free, and
// the compiler can issue the next term's spinor loads before this term's
// arithmetic instead of waiting for each term's loads in turn.
template <int P, int R, int MU, bool FWD, bool DAG, bool STREAM, bool BRANCHLESS = false, typename T>
__device__ __forceinline__ void hop_term_at(Spinor<T>& acc, const char* in, int64_t stride, int nh, const char* lbase,
                                            int64_t lstride, int lpar, int lh, bool cross, C<T> phase) {
    constexpr int EPS = FWD ? (DAG ? 1 : -1) : (DAG ? -1 : 1);
    Spinor<T> v;
    SpinorIO<P>::load(v, in, stride, nh);
    Su3<T> u;
    LinkIO<P, R>::template load<STREAM>(u, lbase, lstride, lpar, MU, lh);
    Half<T> hs, g;
    project_row<MU, EPS, 0>(hs, v);
    project_row<MU, EPS, 1>(hs, v);
    su3_mul<!FWD>(g, u, hs);
    if constexpr (BRANCHLESS) {
        const C<T> f = cross ? phase : C<T>{T(1), T(0)};
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) g.s[r][c] = g.s[r][c] * f;
    } else if (cross) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) g.s[r][c] = g.s[r][c] * phase;
    }
    accumulate_row<MU, EPS, 0>(acc, g);
    accumulate_row<MU, EPS, 1>(acc, g);
}

template <int P, int R, int MU, bool FWD, bool DAG, typename T>
__device__ __forceinline__ void hop_term(Spinor<T>& acc, const HopK& a, const char* in, int link_par,
                                         int link_h, int nh, bool cross, C<T> phase) {
    hop_term_at<P, R, MU, FWD, DAG, true>(acc, in, a.stride, nh, a.gauge, a.gstride, link_par, link_h, cross, phase);
}

// Site decode and the eight neighbour half indices of output site h of parity par.
struct Nbr {
    int f[4], b[4];       // forward / backward neighbour half index per direction
    bool cf[4], cb[4];    // the hop crosses the boundary
};
__device__ __forceinline__ void neighbours(const HopK& a, int par, int h, Nbr& n) {
    const int lxh = a.lxh;
    const int xh = h % lxh;
    int rest = h / lxh;
    const int y = rest % a.L[1];
    rest /= a.L[1];
    const int z = rest % a.L[2];
    const int t = rest / a.L[2];
    const int x = 2 * xh + ((par + y + z + t) & 1);
    const int row = h - xh;
    const int lx = a.L[0];
    const int xf = x + 1 == lx ? 0 : x + 1, xb = x == 0 ? lx - 1 : x - 1;
    n.f[0] = row + (xf >> 1);
    n.b[0] = row + (xb >> 1);
    n.cf[0] = x == lx - 1;
    n.cb[0] = x == 0;
    const int co[4] = {x, y, z, t};
    int st = lxh;
#pragma unroll
    for (int mu = 1; mu < 4; ++mu) {
        const int e = a.L[mu], c = co[mu];
        n.f[mu] = c == e - 1 ? h - (e - 1) * st : h + st;
        n.b[mu] = c == 0 ? h + (e - 1) * st : h - st;
        n.cf[mu] = c == e - 1;
        n.cb[mu] = c == 0;
        st *= e;
    }
}

// The output site h of parity par: the eight terms and the epilogue.  Returns
// this site's contribution to the reduction of the epilogue (0 for kEpiStore).
template <int P, int R, bool DAG, bool OWN, int EPI, int PV>
__device__ __forceinline__ double hop_site(const HopK& a, int par, int h) {
    using T = typename Prec<P>::T;
    const bool two = a.nparity == 2;
    const char* in = a.in + (two ? (int64_t)(1 - par) * a.hbytes : 0);
    double red = 0;
    const int lxh = a.lxh, ly = a.L[1], lz = a.L[2], lt = a.L[3];
    const int xh = h % lxh;
    int rest = h / lxh;
    const int y = rest % ly;
    rest /= ly;
    const int z = rest % lz;
    const int t = rest / lz;
    const int x = 2 * xh + ((par + y + z + t) & 1);
    const int row = h - xh;
    const int opar = 1 - par;

    Spinor<T> acc;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.s[s][c] = {T(0), T(0)};

    // x direction: the neighbour's half index depends on the row parity
    {
        const int lx = a.L[0];
        const int xf = x + 1 == lx ? 0 : x + 1;
        const int xb = x == 0 ? lx - 1 : x - 1;
        const C<T> ph = cvt<T>(a.bc[0]);
        hop_term<P, R, 0, true, DAG>(acc, a, in, par, h, row + (xf >> 1), x == lx - 1, ph);
        const int nb = row + (xb >> 1);
        hop_term<P, R, 0, false, DAG>(acc, a, in, opar, nb, nb, x == 0, conj(ph));
    }
    {
        const int st = lxh;
        const int nf = y == ly - 1 ? h - (ly - 1) * st : h + st;
        const int nb = y == 0 ? h + (ly - 1) * st : h - st;
        const C<T> ph = cvt<T>(a.bc[1]);
        hop_term<P, R, 1, true, DAG>(acc, a, in, par, h, nf, y == ly - 1, ph);
        hop_term<P, R, 1, false, DAG>(acc, a, in, opar, nb, nb, y == 0, conj(ph));
    }
    {
        const int st = lxh * ly;
        const int nf = z == lz - 1 ? h - (lz - 1) * st : h + st;
        const int nb = z == 0 ? h + (lz - 1) * st : h - st;
        const C<T> ph = cvt<T>(a.bc[2]);
        hop_term<P, R, 2, true, DAG>(acc, a, in, par, h, nf, z == lz - 1, ph);
        hop_term<P, R, 2, false, DAG>(acc, a, in, opar, nb, nb, z == 0, conj(ph));
    }
    {
        const int st = lxh * ly * lz;
        const int nf = t == lt - 1 ? h - (lt - 1) * st : h + st;
        const int nb = t == 0 ? h + (lt - 1) * st : h - st;
        const C<T> ph = cvt<T>(a.bc[3]);
        hop_term<P, R, 3, true, DAG>(acc, a, in, par, h, nf, t == lt - 1, ph);
        hop_term<P, R, 3, false, DAG>(acc, a, in, opar, nb, nb, t == 0, conj(ph));
    }

    // epilogue: out = c_hop * acc (+ c_own * own), c = diag(cu, cu, cd, cd)
    const C<T> cuh = cvt<T>(a.cu_hop), cdh = cvt<T>(a.cd_hop);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc.s[0][c] = cuh * acc.s[0][c];
        acc.s[1][c] = cuh * acc.s[1][c];
        acc.s[2][c] = cdh * acc.s[2][c];
        acc.s[3][c] = cdh * acc.s[3][c];
    }
    const int64_t hoff = two ? (int64_t)par * a.hbytes : 0;
    if constexpr (OWN) {
        Spinor<T> o;
        SpinorIO<P>::load(o, a.own + hoff, a.stride, h);
        const C<T> cuo = cvt<T>(a.cu_own), cdo = cvt<T>(a.cd_own);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc.s[0][c] = acc.s[0][c] + cuo * o.s[0][c];
            acc.s[1][c] = acc.s[1][c] + cuo * o.s[1][c];
            acc.s[2][c] = acc.s[2][c] + cdo * o.s[2][c];
            acc.s[3][c] = acc.s[3][c] + cdo * o.s[3][c];
        }
    }
    if constexpr (EPI == kEpiStore || EPI == kEpiStoreNorm) {
        // nontemporal: the launch never reads its output, and kept out of the L2 it
        // leaves it to the neighbour spinors (FP64 24^3 x 48: 101.6 -> 96.8 us; 32^3 x 64:
        // 312 -> 300 us; FP32 and FP16 2-3 % faster).  Storing x and r of the CG update
        // this way as well gained nothing.
        SpinorIO<P>::template store<true>(a.out + hoff, a.stride, h, acc);
        if constexpr (EPI == kEpiStoreNorm) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) red += (double)norm2(acc.s[s][c]);
        }
    } else {
        // r -= alpha (A p); the CG solvers update x in their p = r + beta p launch,
        // which reads p anyway
        const T alpha = (T)a.st->alpha;
        const int64_t voff = two ? (int64_t)par * a.vhbytes : 0;
        Spinor<T> rv;
        SpinorIO<PV>::load(rv, a.r + voff, a.stride, h);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) rv.s[s][c] = rv.s[s][c] - scale(alpha, acc.s[s][c]);
        SpinorIO<PV>::store(a.r + voff, a.stride, h, rv);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) red += (double)norm2(rv.s[s][c]);
    }
    return red;
}

// First pass of the epilogue's reduction: this block's sum to partials[tile].
// The solver scalars are finished by the launch that follows (cg_finish).
template <int EPI, int BS = kBlock>
__device__ __forceinline__ void hop_reduce(const HopK& a, double red, int tile) {
    if constexpr (EPI != kEpiStore) {
        const double v[1] = {red};
        block_partial<1, BS>(v, a.partials, tile);
    }
}

// Column-order regions: square (y, z) tiles of side b dividing both extents,
// no larger than the L2 allows for the fields swept (two slices of a region
// for every right-hand side in flight within about 3 MB), with at least 8
// regions; among those the most even split over the 8 XCDs, then the largest.
inline void column_regions(const HopParams& a, HopK& k) {
    const int sb = a.prec == TMQCD_F64 ? 192 : (a.prec == TMQCD_F32 ? 96 : 52);
    const int64_t target = (int64_t)3 << 20;
    const int ly = a.g.L[1], lz = a.g.L[2], lxh = a.g.lxh, nr = a.nrhs > 1 ? a.nrhs : 1;
    int best = 1;
    double best_imb = 1e30;
    for (int b = 2; b <= ly && b <= lz; ++b) {
        if (ly % b || lz % b) continue;
        const int nreg = (ly / b) * (lz / b);
        const int64_t window = 2LL * lxh * b * b * nr * sb;
        if (nreg < kNumXcd || window > target) continue;
        const double imb = (double)(((nreg + kNumXcd - 1) / kNumXcd) * kNumXcd) / nreg;
        if (imb <= best_imb) {
            best = b;
            best_imb = imb;
        }
    }
    k.by = k.bz = best;
    k.nry = (ly + best - 1) / best;
    k.nreg = k.nry * ((lz + best - 1) / best);
}

// w: output sites per block (the block size, or 64 for the multi-RHS kernel)
inline HopK make_hopk(const HopParams& a, int w) {
    HopK k;
    k.gauge = static_cast<const char*>(a.gauge);
    k.in = static_cast<const char*>(a.in);
    k.own = static_cast<const char*>(a.own);
    k.out = static_cast<char*>(a.out);
    k.r = static_cast<char*>(a.r);
    k.st = a.st;
    k.partials = a.partials;
    k.stride = a.g.stride;
    k.gstride = a.g.gstride;
    k.hbytes = half_field_bytes(a.g, a.prec);
    k.vhbytes = half_field_bytes(a.g, a.vprec);
    for (int i = 0; i < 4; ++i) {
        k.L[i] = a.g.L[i];
        k.bc[i] = {a.bc[i].re, a.bc[i].im};
    }
    k.lxh = a.g.lxh;
    k.vh = (int)a.g.vh;
    k.order = a.order;
    k.width = w;
    k.fin_partials = a.fin_partials;
    k.fin_n = a.fin_n;
    k.fin_kind = a.fin_kind;
    k.lt = a.g.L[3];
    k.slice = (int)(a.g.vh / a.g.L[3]);
    k.nz = a.order == kOrderSlabT2 ? 4 : (a.order == kOrderSlabT4 ? 2 : kNumXcd);
    const int nt = kNumXcd / k.nz;
    k.tlen = (k.lt + nt - 1) / nt;
    k.q = (k.slice + k.nz - 1) / k.nz;
    k.tq = (k.q + w - 1) / w;
    column_regions(a, k);
    if (slab_order(a.order)) k.nb_half = kNumXcd * k.tlen * k.tq;
    else if (a.order == kOrderColumn) {
        const int tqc = (k.lxh * k.by * k.bz + w - 1) / w;
        k.nb_half = kNumXcd * ((k.nreg + kNumXcd - 1) / kNumXcd) * k.lt * tqc;
        k.tq = tqc;
    } else k.nb_half = (int)((a.g.vh + w - 1) / w);
    k.nblocks = a.nparity * k.nb_half;
    k.out_parity = a.out_parity;
    k.nparity = a.nparity;
    k.cu_own = {a.cu_own.re, a.cu_own.im};
    k.cd_own = {a.cd_own.re, a.cd_own.im};
    k.cu_hop = {a.cu_hop.re, a.cu_hop.im};
    k.cd_hop = {a.cd_hop.re, a.cd_hop.im};
    return k;
}

// Multi-RHS launch (nrhs > 1, store epilogue only), any precision and link format.
hipError_t launch_hop_mrhs(const HopParams& a, const HopK& k, hipStream_t s);

}  // namespace stencil
}  // namespace tmqcd
