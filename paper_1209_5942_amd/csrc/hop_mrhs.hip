// Multi-RHS hop (several right-hand sides share every link load).
#include "stencil.h"

namespace tmqcd {
namespace stencil {
namespace {

// Multi-RHS hop: a block owns 64 output sites and a group of right-hand sides;
// its four waves first copy the eight links of those sites into LDS (read from
// HBM once per group), then loop over the group, wave w handling its rhs w,
// w+4, w+8, ...  Blocks [g*tiles, (g+1)*tiles) serve group g, so the whole
// lattice is swept once per group: fewer fields in flight per sweep keep more
// of their t-neighbours in the L2, at the price of re-reading the links.
// Fields of consecutive right-hand sides are `*_fstride` bytes apart.
//
// Inside the multi-RHS CG (FP64) the launch also carries one solver state per
// column: columns whose solve has stopped are skipped (a column belongs to one
// wave at a time, so the test is wave-uniform), and the epilogues of the CG
// stages run per column: kEpiStoreNorm stores the output and sums its |out|^2,
// kEpiCgUpdate updates r -= alpha out and sums |r|^2 (x += alpha p is left to
// the search-direction update, which reads p anyway); the sums of a wave's 64
// sites go to partials[column * tiles + tile] (no block-level step).
struct MrhsK {
    int nrhs, group, tiles;
    int64_t in_fstride, own_fstride, out_fstride;
    const CgState* st;       // per column, or nullptr outside CG
    double* partials;        // [nrhs][tiles]
    char* r;                 // CG update: r (FP64), fields v_fstride apart
    int64_t v_fstride;
};

template <int P, int R, bool DAG, bool OWN, int EPI>
__global__ __launch_bounds__(kBlock) void hop_mrhs_kernel(const HopK a, const MrhsK m) {
    using T = typename Prec<P>::T;
    using LIO = LinkIO<P, R>;
    using Unit = typename LIO::Unit;
    constexpr int NU = LIO::kUnits;
    __shared__ Unit tile[8 * NU * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = blockIdx.x / m.tiles;
    int par, h;
    const bool valid = block_site(a, blockIdx.x - g * m.tiles, lane, par, h);
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
    if (EPI == kEpiStore && !valid) return;   // the reducing epilogues keep every lane for the wave sums
    const char* lt = reinterpret_cast<const char*>(tile);
    const C<T> cuh = cvt<T>(a.cu_hop), cdh = cvt<T>(a.cd_hop);
    const int64_t hoff = two ? (int64_t)par * a.hbytes : 0;
    const int64_t ioff = two ? (int64_t)(1 - par) * a.hbytes : 0;
    const int rend = min(m.nrhs, (g + 1) * m.group);
    const int tile_id = blockIdx.x - g * m.tiles;
#pragma unroll 1
    for (int r = g * m.group + wave; r < rend; r += kWaves) {
        if (m.st != nullptr && m.st[r].done) continue;   // this column's solve has stopped
        // The link reads from the tile do not depend on r; without this barrier
        // the compiler hoists all eight links out of the loop into registers.
        __asm__ volatile("" ::: "memory");
        double red = 0.0;
        if (valid) {
        const char* in = a.in + r * m.in_fstride + ioff;
        Spinor<T> acc;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc.s[s][c] = {T(0), T(0)};
#define TMQCD_TERMS(MU)                                                                                     \
    {                                                                                                       \
        const C<T> ph = cvt<T>(a.bc[MU]);                                                                   \
        hop_term_at<P, R, MU, true, DAG, false, true>(acc, in, a.stride, n.f[MU], lt, 64, 0, lane, n.cf[MU], ph);  \
        hop_term_at<P, R, MU, false, DAG, false, true>(acc, in, a.stride, n.b[MU], lt, 64, 1, lane, n.cb[MU],      \
                                                       conj(ph));                                                  \
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
        if constexpr (EPI == kEpiStore) {
            SpinorIO<P>::template store<true>(a.out + r * m.out_fstride + hoff, a.stride, h, acc);
        } else if constexpr (EPI == kEpiStoreNorm) {
            SpinorIO<P>::template store<true>(a.out + r * m.out_fstride + hoff, a.stride, h, acc);   // not read by this launch
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) red += (double)norm2(acc.s[s][c]);
        } else {
            static_assert(P == TMQCD_F64, "the multi-RHS CG update runs in FP64");
            const T alpha = (T)m.st[r].alpha;
            const int64_t voff = two ? (int64_t)par * a.vhbytes : 0;
            Spinor<T> rv;
            SpinorIO<P>::load(rv, m.r + r * m.v_fstride + voff, a.stride, h);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    rv.s[s][c] = rv.s[s][c] - scale(alpha, acc.s[s][c]);
                    red += (double)norm2(rv.s[s][c]);
                }
            SpinorIO<P>::store(m.r + r * m.v_fstride + voff, a.stride, h, rv);
        }
        }   // valid
        if constexpr (EPI != kEpiStore) {
            red = wave_sum(red);
            if (lane == 0) m.partials[(int64_t)r * m.tiles + tile_id] = red;
        }
    }
}

template <int P, int R>
hipError_t launch_mrhs(const HopParams& a, const HopK& k, hipStream_t s) {
    MrhsK m;
    m.nrhs = a.nrhs;
    m.group = a.group > 0 && a.group < a.nrhs ? a.group : a.nrhs;
    m.tiles = k.nblocks;
    m.in_fstride = a.in_fstride;
    m.own_fstride = a.own_fstride;
    m.out_fstride = a.out_fstride;
    m.st = a.st;
    m.partials = a.partials;
    m.r = static_cast<char*>(a.r);
    m.v_fstride = a.v_fstride;
    const bool own = a.own != nullptr;
    const dim3 grid(k.nblocks * ((m.nrhs + m.group - 1) / m.group)), block(kBlock);
    if (a.epi == kEpiStore) {
        if (!a.dag && !own) hipLaunchKernelGGL((hop_mrhs_kernel<P, R, false, false, kEpiStore>), grid, block, 0, s, k, m);
        else if (a.dag && !own) hipLaunchKernelGGL((hop_mrhs_kernel<P, R, true, false, kEpiStore>), grid, block, 0, s, k, m);
        else if (!a.dag && own) hipLaunchKernelGGL((hop_mrhs_kernel<P, R, false, true, kEpiStore>), grid, block, 0, s, k, m);
        else hipLaunchKernelGGL((hop_mrhs_kernel<P, R, true, true, kEpiStore>), grid, block, 0, s, k, m);
        return hipGetLastError();
    }
    // the CG stages (FP64): store + |out|^2 of A p (no dagger, own term), update after A^+ (dagger, own term)
    if constexpr (P == TMQCD_F64) {
        if (a.st == nullptr || a.partials == nullptr || !own) return hipErrorInvalidValue;
        if (a.epi == kEpiStoreNorm && !a.dag)
            hipLaunchKernelGGL((hop_mrhs_kernel<P, R, false, true, kEpiStoreNorm>), grid, block, 0, s, k, m);
        else if (a.epi == kEpiCgUpdate && a.dag && a.r)
            hipLaunchKernelGGL((hop_mrhs_kernel<P, R, true, true, kEpiCgUpdate>), grid, block, 0, s, k, m);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_hop_mrhs(const HopParams& a, const HopK& k, hipStream_t s) {
    return with_link_format(a.prec, a.recon, [&](auto p, auto r) {
        return launch_mrhs<decltype(p)::value, decltype(r)::value>(a, k, s);
    });
}

}  // namespace stencil
}  // namespace tmqcd
