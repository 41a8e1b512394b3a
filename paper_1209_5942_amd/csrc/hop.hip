// The even-odd hop stencil (paper, section 2.1: the hopping part of D_tm, and the
// storage-format section for the parity-split SoA layout).
//
// One thread per output site.  For each of the 8 directions the neighbour
// spinor is spin-projected to a half spinor with (1 -+ gamma_mu), multiplied by
// U_mu(x) or U_mu(x - mu)^+, and the lower spin components are rebuilt from the
// upper ones (the projectors have rank 2), which gives the standard 1320 flops
// per site.  The epilogue applies the twisted diagonal and, inside CG, the
// solver update and a deterministic FP64 reduction.
#include "device.h"
#include "internal.h"

namespace tmqcd {
namespace {

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
    char* x;
    char* r;
    const char* p;
    CgState* st;
    double* partials;
    int64_t stride, gstride, hbytes, vhbytes;
    int L[4];
    int lxh, vh, nb_half, nblocks, out_parity, nparity, swizzle;
    C<double> bc[4];
    C<double> cu_own, cd_own, cu_hop, cd_hop;
};

// One of the eight terms: FWD: b+ (1 -+ gamma_mu) U_mu(x) psi(x+mu);
// backward: b- (1 +- gamma_mu) U_mu(x-mu)^+ psi(x-mu) (signs flip for H^+).
// The link is read from `lbase` in the packed link layout with stride
// `lstride` (global memory, or a block's link tile in LDS).
template <int P, int R, int MU, bool FWD, bool DAG, bool STREAM, typename T>
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
    if (cross) {
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
            SpinorIO<P>::store(a.out + hoff, a.stride, h, acc);
            if constexpr (EPI == kEpiStoreNorm) {
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int c = 0; c < 3; ++c) red += (double)norm2(acc.s[s][c]);
            }
        } else {
            // x += alpha p, r -= alpha (A p)
            const T alpha = (T)a.st->alpha;
            const int64_t voff = two ? (int64_t)par * a.vhbytes : 0;
            Spinor<T> pv, xv, rv;
            SpinorIO<P>::load(pv, a.p + hoff, a.stride, h);
            SpinorIO<PV>::load(xv, a.x + voff, a.stride, h);
            SpinorIO<PV>::load(rv, a.r + voff, a.stride, h);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xv.s[s][c] = xv.s[s][c] + scale(alpha, pv.s[s][c]);
                    rv.s[s][c] = rv.s[s][c] - scale(alpha, acc.s[s][c]);
                }
            SpinorIO<PV>::store(a.x + voff, a.stride, h, xv);
            SpinorIO<PV>::store(a.r + voff, a.stride, h, rv);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) red += (double)norm2(rv.s[s][c]);
        }
    return red;
}

// Grid reduction of the epilogue's per-site values and the solver-scalar
// update by the last tile to finish (tile: this block's logical index).
template <int EPI, int BS = kBlock>
__device__ __forceinline__ void hop_reduce(const HopK& a, double red, int tile, int ntiles) {
    if constexpr (EPI != kEpiStore) {
        double v[1] = {red}, tot[1];
        const int slot = EPI == kEpiStoreNorm ? 0 : 1;
        if (grid_reduce<1, BS>(v, tot, a.partials, &a.st->counter[slot], tile, ntiles) && threadIdx.x == 0) {
            CgState* st = a.st;
            if constexpr (EPI == kEpiStoreNorm) {
                const double pap = tot[0];
                st->pAp = pap;
                if (!(pap > 0.0) || !isfinite(pap)) st->done = kDoneBreakdown;
                else st->alpha = st->rr / pap;
            } else {
                const double rr = tot[0];
                const double rr_old = st->rr;
                st->rr_prev = rr_old;
                st->rr = rr;
                st->beta = rr / rr_old;
                const int it = st->iter + 1;
                st->iter = it;
                if (!isfinite(rr)) st->done = kDoneBreakdown;
                else if (rr <= st->stop_rr || it >= st->cycle_end) st->done = kDoneStop;
                else if (it >= st->max_iter) st->done = kDoneMaxIter;
            }
        }
    }
}

// BS threads per block (a tuning choice); with a.swizzle the block index is
// remapped so that each XCD works on a contiguous range of sites.
template <int P, int R, bool DAG, bool OWN, int EPI, int PV, int BS>
__global__ __launch_bounds__(BS) void hop_kernel(const HopK a) {
    static_assert(std::is_same<typename Prec<P>::T, typename Prec<PV>::T>::value,
                  "vector and dslash compute types differ");
    if constexpr (EPI != kEpiStore) {
        if (a.st->done) return;
    }
    const int bid = a.swizzle ? xcd_swizzle(blockIdx.x, a.nblocks) : (int)blockIdx.x;
    int par = a.out_parity, lb = bid;
    if (a.nparity == 2) {
        par = bid >= a.nb_half ? 1 : 0;
        lb = bid - par * a.nb_half;
    }
    const int h = lb * BS + threadIdx.x;
    const double red = h < a.vh ? hop_site<P, R, DAG, OWN, EPI, PV>(a, par, h) : 0.0;
    hop_reduce<EPI, BS>(a, red, bid, a.nblocks);
}

// Several lattices in one launch: a grid-stride loop over the tiles of all
// lattices (tile_start[i] is the first tile of lattice i).  Lattices whose
// solver has stopped are skipped; each lattice reduces into its own state.
constexpr int kMaxBatch = 8;
struct HopBatch {
    int n;
    int tile_start[kMaxBatch + 1];
    HopK lat[kMaxBatch];
};

template <int P, int R, bool DAG, bool OWN, int EPI, int PV>
__global__ __launch_bounds__(kBlock) void hop_batch_kernel(const HopBatch b) {
    const int total = b.tile_start[b.n];
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        int i = 0;
        while (tile >= b.tile_start[i + 1]) ++i;
        const HopK& a = b.lat[i];
        if constexpr (EPI != kEpiStore) {
            if (a.st->done) continue;
        }
        const int lt = tile - b.tile_start[i];
        int par = a.out_parity, lb = lt;
        if (a.nparity == 2) {
            par = lt >= a.nb_half ? 1 : 0;
            lb = lt - par * a.nb_half;
        }
        const int h = lb * kBlock + threadIdx.x;
        const double red = h < a.vh ? hop_site<P, R, DAG, OWN, EPI, PV>(a, par, h) : 0.0;
        hop_reduce<EPI>(a, red, lt, a.nblocks);
    }
}

// Multi-RHS hop: a block owns 64 output sites; its four waves first copy the
// eight links of those sites into LDS (each link read from HBM once), then
// loop over the right-hand sides, wave w handling rhs w, w+4, w+8, ...
// Fields of consecutive right-hand sides are `*_fstride` bytes apart.
struct MrhsK {
    int nrhs, nb_half, nblocks;
    int64_t in_fstride, own_fstride, out_fstride;
};

template <int P, int R, bool DAG, bool OWN>
__global__ __launch_bounds__(kBlock) void hop_mrhs_kernel(const HopK a, const MrhsK m) {
    using T = typename Prec<P>::T;
    using LIO = LinkIO<P, R>;
    using Unit = typename LIO::Unit;
    constexpr int NU = LIO::kUnits;
    __shared__ Unit tile[8 * NU * 64];
    const int bid = xcd_swizzle(blockIdx.x, m.nblocks);
    int par = a.out_parity, lb = bid;
    if (a.nparity == 2) {
        par = bid >= m.nb_half ? 1 : 0;
        lb = bid - par * m.nb_half;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lb * 64 + lane;
    const bool valid = h < a.vh;
    const bool two = a.nparity == 2;
    Nbr n;
    if (valid) {
        neighbours(a, par, h, n);
        // links 0..3: U_mu(x) (parity par, index h); 4..7: U_mu(x - mu) (other parity)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int l = 2 * wave + q;
            const int mu = l & 3;
            const int lp = l < 4 ? par : 1 - par;
            // select, not an indexed load: a private array indexed at run time would live in scratch
            const int nbm = mu == 0 ? n.b[0] : mu == 1 ? n.b[1] : mu == 2 ? n.b[2] : n.b[3];
            const int lh = l < 4 ? h : nbm;
            const Unit* src = reinterpret_cast<const Unit*>(a.gauge) + (int64_t)((lp * 4 + mu) * NU) * a.gstride + lh;
#pragma unroll
            for (int k = 0; k < NU; ++k) tile[(l * NU + k) * 64 + lane] = ld_stream(src + k * a.gstride);
        }
    }
    __syncthreads();
    if (!valid) return;
    const char* lt = reinterpret_cast<const char*>(tile);
    const C<T> cuh = cvt<T>(a.cu_hop), cdh = cvt<T>(a.cd_hop);
    const int64_t hoff = two ? (int64_t)par * a.hbytes : 0;
    const int64_t ioff = two ? (int64_t)(1 - par) * a.hbytes : 0;
#pragma unroll 1
    for (int r = wave; r < m.nrhs; r += kWaves) {
        // The link reads from the tile do not depend on r; without this barrier
        // the compiler hoists all eight links out of the loop into registers.
        __asm__ volatile("" ::: "memory");
        const char* in = a.in + r * m.in_fstride + ioff;
        Spinor<T> acc;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc.s[s][c] = {T(0), T(0)};
#define TMQCD_TERMS(MU)                                                                                     \
    {                                                                                                       \
        const C<T> ph = cvt<T>(a.bc[MU]);                                                                   \
        hop_term_at<P, R, MU, true, DAG, false>(acc, in, a.stride, n.f[MU], lt, 64, 0, lane, n.cf[MU], ph);       \
        hop_term_at<P, R, MU, false, DAG, false>(acc, in, a.stride, n.b[MU], lt, 64, 1, lane, n.cb[MU], conj(ph)); \
    }
        TMQCD_TERMS(0)
        TMQCD_TERMS(1)
        TMQCD_TERMS(2)
        TMQCD_TERMS(3)
#undef TMQCD_TERMS
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc.s[0][c] = cuh * acc.s[0][c];
            acc.s[1][c] = cuh * acc.s[1][c];
            acc.s[2][c] = cdh * acc.s[2][c];
            acc.s[3][c] = cdh * acc.s[3][c];
        }
        if constexpr (OWN) {
            Spinor<T> o;
            SpinorIO<P>::load(o, a.own + r * m.own_fstride + hoff, a.stride, h);
            const C<T> cuo = cvt<T>(a.cu_own), cdo = cvt<T>(a.cd_own);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc.s[0][c] = acc.s[0][c] + cuo * o.s[0][c];
                acc.s[1][c] = acc.s[1][c] + cuo * o.s[1][c];
                acc.s[2][c] = acc.s[2][c] + cdo * o.s[2][c];
                acc.s[3][c] = acc.s[3][c] + cdo * o.s[3][c];
            }
        }
        SpinorIO<P>::store(a.out + r * m.out_fstride + hoff, a.stride, h, acc);
    }
}

template <int P, int R>
hipError_t launch_mrhs(const HopParams& a, const HopK& k, hipStream_t s) {
    MrhsK m;
    m.nrhs = a.nrhs;
    m.nb_half = (int)((a.g.vh + 63) / 64);
    m.nblocks = a.nparity * m.nb_half;
    m.in_fstride = a.in_fstride;
    m.own_fstride = a.own_fstride;
    m.out_fstride = a.out_fstride;
    const bool own = a.own != nullptr;
    const dim3 grid(m.nblocks), block(kBlock);
    if (!a.dag && !own) hipLaunchKernelGGL((hop_mrhs_kernel<P, R, false, false>), grid, block, 0, s, k, m);
    else if (a.dag && !own) hipLaunchKernelGGL((hop_mrhs_kernel<P, R, true, false>), grid, block, 0, s, k, m);
    else if (!a.dag && own) hipLaunchKernelGGL((hop_mrhs_kernel<P, R, false, true>), grid, block, 0, s, k, m);
    else hipLaunchKernelGGL((hop_mrhs_kernel<P, R, true, true>), grid, block, 0, s, k, m);
    return hipGetLastError();
}

template <int P, int R, bool DAG, bool OWN, int EPI>
hipError_t launch_inst(const HopK& k, int block, hipStream_t s) {
    constexpr int PV = P == TMQCD_F64 ? TMQCD_F64 : TMQCD_F32;
    if (block == 128)
        hipLaunchKernelGGL((hop_kernel<P, R, DAG, OWN, EPI, PV, 128>), dim3(k.nblocks), dim3(128), 0, s, k);
    else
        hipLaunchKernelGGL((hop_kernel<P, R, DAG, OWN, EPI, PV, 256>), dim3(k.nblocks), dim3(256), 0, s, k);
    return hipGetLastError();
}

template <int P, int R>
hipError_t dispatch_variant(const HopParams& a, const HopK& k, hipStream_t s) {
    if (a.nrhs > 1) return a.epi == kEpiStore ? launch_mrhs<P, R>(a, k, s) : hipErrorInvalidValue;
    const bool own = a.own != nullptr;
    switch (a.epi) {
        case kEpiStore:
            if (!a.dag && !own) return launch_inst<P, R, false, false, kEpiStore>(k, a.block, s);
            if (a.dag && !own) return launch_inst<P, R, true, false, kEpiStore>(k, a.block, s);
            if (!a.dag && own) return launch_inst<P, R, false, true, kEpiStore>(k, a.block, s);
            return launch_inst<P, R, true, true, kEpiStore>(k, a.block, s);
        case kEpiStoreNorm:
            if (!a.dag && own) return launch_inst<P, R, false, true, kEpiStoreNorm>(k, a.block, s);
            break;
        case kEpiCgUpdate:
            if (a.dag && own) return launch_inst<P, R, true, true, kEpiCgUpdate>(k, a.block, s);
            break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

int hop_blocks(const Geom& g, int nparity) { return nparity * (int)((g.vh + kMinBlock - 1) / kMinBlock); }

static HopK make_hopk(const HopParams& a) {
    HopK k;
    k.gauge = static_cast<const char*>(a.gauge);
    k.in = static_cast<const char*>(a.in);
    k.own = static_cast<const char*>(a.own);
    k.out = static_cast<char*>(a.out);
    k.x = static_cast<char*>(a.x);
    k.r = static_cast<char*>(a.r);
    k.p = static_cast<const char*>(a.p);
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
    const int bs = a.block == 128 ? 128 : 256;
    k.nb_half = (int)((a.g.vh + bs - 1) / bs);
    k.nblocks = a.nparity * k.nb_half;
    k.swizzle = a.swizzle;
    k.out_parity = a.out_parity;
    k.nparity = a.nparity;
    k.cu_own = {a.cu_own.re, a.cu_own.im};
    k.cd_own = {a.cd_own.re, a.cd_own.im};
    k.cu_hop = {a.cu_hop.re, a.cu_hop.im};
    k.cd_hop = {a.cd_hop.re, a.cd_hop.im};
    return k;
}

hipError_t launch_hop(const HopParams& a_in, hipStream_t s) {
    HopParams a = a_in;
    if (a.block == 0) {   // not chosen by the caller: the tuned choice, else 256 threads with the XCD remap
        TuneChoice t;
        if (a.nrhs <= 1 && tune_lookup(a, &t)) {
            a.block = t.block;
            a.swizzle = t.swizzle;
        } else {
            a.block = 256;
            a.swizzle = 1;
        }
    }
    const HopK k = make_hopk(a);
    const int want_vprec = a.prec == TMQCD_F64 ? TMQCD_F64 : TMQCD_F32;
    if (a.epi == kEpiCgUpdate && a.vprec != want_vprec) return hipErrorInvalidValue;
    const bool r12 = a.recon == TMQCD_RECON12;
    switch (a.prec) {
        case TMQCD_F64:
            return r12 ? dispatch_variant<TMQCD_F64, TMQCD_RECON12>(a, k, s)
                       : dispatch_variant<TMQCD_F64, TMQCD_RECON18>(a, k, s);
        case TMQCD_F32:
            return r12 ? dispatch_variant<TMQCD_F32, TMQCD_RECON12>(a, k, s)
                       : dispatch_variant<TMQCD_F32, TMQCD_RECON18>(a, k, s);
        case TMQCD_F16:
            return r12 ? dispatch_variant<TMQCD_F16, TMQCD_RECON12>(a, k, s)
                       : dispatch_variant<TMQCD_F16, TMQCD_RECON18>(a, k, s);
    }
    return hipErrorInvalidValue;
}

namespace {
template <bool DAG, bool OWN, int EPI>
hipError_t launch_batch_inst(const HopBatch& b, int grid, hipStream_t s) {
    hipLaunchKernelGGL((hop_batch_kernel<TMQCD_F64, TMQCD_RECON18, DAG, OWN, EPI, TMQCD_F64>), dim3(grid),
                       dim3(kBlock), 0, s, b);
    return hipGetLastError();
}
template <bool DAG, bool OWN, int EPI>
hipError_t launch_batch_inst12(const HopBatch& b, int grid, hipStream_t s) {
    hipLaunchKernelGGL((hop_batch_kernel<TMQCD_F64, TMQCD_RECON12, DAG, OWN, EPI, TMQCD_F64>), dim3(grid),
                       dim3(kBlock), 0, s, b);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_hop_batch(const HopParams* ps, int n, int max_grid, hipStream_t s) {
    if (n < 1 || n > kMaxBatch) return hipErrorInvalidValue;
    HopBatch b;
    b.n = n;
    b.tile_start[0] = 0;
    for (int i = 0; i < n; ++i) {
        const HopParams& a = ps[i];
        if (a.prec != TMQCD_F64 || a.vprec != TMQCD_F64 || a.nrhs > 1 || a.recon != ps[0].recon ||
            a.dag != ps[0].dag || (a.own != nullptr) != (ps[0].own != nullptr) || a.epi != ps[0].epi)
            return hipErrorInvalidValue;
        HopParams a256 = a;
        a256.block = 256;
        b.lat[i] = make_hopk(a256);
        b.tile_start[i + 1] = b.tile_start[i] + b.lat[i].nblocks;
    }
    const int total = b.tile_start[n];
    const int grid = total < max_grid ? total : max_grid;
    const HopParams& a = ps[0];
    const bool own = a.own != nullptr, r12 = a.recon == TMQCD_RECON12;
#define TMQCD_BATCH(D, O, E) return r12 ? launch_batch_inst12<D, O, E>(b, grid, s) : launch_batch_inst<D, O, E>(b, grid, s)
    switch (a.epi) {
        case kEpiStore:
            if (!a.dag && !own) TMQCD_BATCH(false, false, kEpiStore);
            if (a.dag && !own) TMQCD_BATCH(true, false, kEpiStore);
            if (!a.dag && own) TMQCD_BATCH(false, true, kEpiStore);
            TMQCD_BATCH(true, true, kEpiStore);
        case kEpiStoreNorm:
            if (!a.dag && own) TMQCD_BATCH(false, true, kEpiStoreNorm);
            break;
        case kEpiCgUpdate:
            if (a.dag && own) TMQCD_BATCH(true, true, kEpiCgUpdate);
            break;
    }
#undef TMQCD_BATCH
    return hipErrorInvalidValue;
}

}  // namespace tmqcd
