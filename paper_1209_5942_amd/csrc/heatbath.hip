// Pure-gauge heatbath and overrelaxation on the Wilson plaquette action (the
// paper's heatbath section: SU(3) updated through its three SU(2) subgroups by
// project / update / extend), on FP64 or FP32 links with arithmetic to match
// (the paper measures its heatbath in single precision).  One launch updates the links U_mu(x) of one
// direction and one parity: their staples hold no link of that set, so the
// threads are independent.  Per link, with V the staple sum (the plaquettes
// through the link sum to Re Tr[U V]) and W = U V:
//   for the subgroups (0,1), (0,2), (1,2): the quaternion part of W's 2x2 block,
//   q = k s (s in SU(2)); heatbath: r = x s^+ with x in SU(2) of weight
//   exp(alpha x0), alpha = (2/3) beta k; overrelaxation: r = (s^+)^2, which
//   keeps Re Tr[U V]; then U <- R U and W <- R W (R = r on the subgroup's rows).
// x0 has density sqrt(1 - x0^2) exp(alpha x0): below alpha = 2 by inverting the
// exponential and accepting with sqrt(1 - x0^2), above by Kennedy and
// Pendleton's method.  Random numbers come from Philox4x32-10 (Salmon et al.,
// SC'11) with key = seed and counter = (4 s + mu, sweep, subgroup * 2^16 +
// trial, 0), s the canonical site index; the direction of x uses trial 0xFFFF.
#include <cstdint>

#include "device.h"
#include "internal.h"
#include "su3.h"
#include "stencil.h"

namespace tmqcd {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;
constexpr uint32_t kDirTrial = 0xFFFFu;
constexpr uint32_t kMaxTrials = 0xFFFEu;
constexpr double kAlphaSwitch = 2.0;

// Philox4x32-10: ten rounds, the key raised by the Weyl constants between rounds
__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t lo0 = kPhiloxM0 * c[0], hi0 = __umulhi(kPhiloxM0, c[0]);
        const uint32_t lo1 = kPhiloxM1 * c[2], hi1 = __umulhi(kPhiloxM1, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
}

__device__ __forceinline__ double unit(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

struct Rng {
    uint32_t k0, k1, link, sweep;
    // the four words of one counter as uniforms in (0, 1) (formed in FP64, then rounded to T)
    template <typename T>
    __device__ __forceinline__ void words(uint32_t sub, uint32_t trial, T u[4]) const {
        uint32_t c[4] = {link, sweep, (sub << 16) + trial, 0u};
        philox(c, k0, k1);
#pragma unroll
        for (int i = 0; i < 4; ++i) u[i] = (T)unit(c[i]);
    }
};

// x0 in [-1, 1] with density sqrt(1 - x0^2) exp(alpha x0), in the arithmetic type T
template <typename T>
__device__ T sample_x0(T alpha, const Rng& g, uint32_t sub) {
    const T pi = T(M_PI);
    for (uint32_t trial = 0; trial < kMaxTrials; ++trial) {
        T u[4];
        g.words(sub, trial, u);
        if (alpha < T(kAlphaSwitch)) {
            const T x = alpha > T(0) ? T(-1) + log1p(u[0] * expm1(T(2) * alpha)) / alpha : T(2) * u[0] - T(1);
            if (u[1] <= sqrt(fmax(T(0), (T(1) - x) * (T(1) + x)))) return x;
        } else {
            const T cs = cos(T(2) * pi * u[1]);
            const T lam2 = -(log(u[0]) + cs * cs * log(u[2])) / (T(2) * alpha);
            if (u[3] * u[3] <= T(1) - lam2) return T(1) - T(2) * lam2;
        }
    }
    return T(1);   // unreachable in practice: every method accepts with probability above one half
}

// rows a and b of m <- r (2x2) applied to those rows
template <typename T>
__device__ __forceinline__ void rotate_rows(Su3<T>& m, int a, int b, const C<T> r[2][2]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const C<T> ma = m.m[a][j], mb = m.m[b][j];
        m.m[a][j] = r[0][0] * ma + r[0][1] * mb;
        m.m[b][j] = r[1][0] * ma + r[1][1] * mb;
    }
}

template <int A, int B, typename T>
__device__ __forceinline__ void subgroup(Su3<T>& u, Su3<T>& w, bool heatbath, T beta, const Rng& g, uint32_t sub) {
    const C<T> w00 = w.m[A][A], w01 = w.m[A][B], w10 = w.m[B][A], w11 = w.m[B][B];
    T a0 = T(0.5) * (w00.re + w11.re), a1 = T(0.5) * (w01.im + w10.im);
    T a2 = T(0.5) * (w01.re - w10.re), a3 = T(0.5) * (w00.im - w11.im);
    const T kk = sqrt(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3);
    if (kk > T(0)) {
        a0 /= kk;
        a1 /= kk;
        a2 /= kk;
        a3 /= kk;
    } else {
        a0 = T(1);
        a1 = a2 = a3 = T(0);
    }
    // s^+ = a0 - i a.sigma
    const C<T> sd[2][2] = {{{a0, -a3}, {-a2, -a1}}, {{a2, -a1}, {a0, a3}}};
    C<T> r[2][2];
    if (heatbath) {
        const T x0 = sample_x0<T>(T(2.0 / 3.0) * beta * kk, g, sub);
        T ud[4];
        g.words(sub, kDirTrial, ud);
        const T cth = T(2) * ud[0] - T(1);
        const T phi = T(2) * T(M_PI) * ud[1];
        // (1 - x)(1 + x), not 1 - x x: accurate near x = +-1, where the root magnifies rounding
        const T rad = sqrt(fmax(T(0), (T(1) - x0) * (T(1) + x0)));
        const T sth = sqrt(fmax(T(0), (T(1) - cth) * (T(1) + cth)));
        const T x1 = rad * sth * cos(phi), x2 = rad * sth * sin(phi), x3 = rad * cth;
        const C<T> x[2][2] = {{{x0, x3}, {x2, x1}}, {{-x2, x1}, {x0, -x3}}};
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) r[i][j] = x[i][0] * sd[0][j] + x[i][1] * sd[1][j];
    } else if (kk > T(0)) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) r[i][j] = sd[i][0] * sd[0][j] + sd[i][1] * sd[1][j];
    } else {
        return;
    }
    rotate_rows(u, A, B, r);
    rotate_rows(w, A, B, r);
}

// map: which sites of parity par a block covers (the hop's t-slab order: each XCD walks its eighth
// of every t-slice through all t, so the links around the next slice are in its L2 already; 12 %
// faster for the heatbath and 21 % for overrelaxation than consecutive blocks at 24^3 x 48)
// P: link storage (FP64 or FP32 RECON18); the arithmetic is FP64 or FP32 accordingly
template <int P>
__global__ __launch_bounds__(kBlock) void su3_update_kernel(LatK k, stencil::HopK map, char* gauge, int mu, int par,
                                                            double beta, uint32_t key0, uint32_t key1, uint32_t sweep,
                                                            int heatbath) {
    using T = typename Prec<P>::T;
    int pp, h;
    if (!stencil::block_site(map, blockIdx.x, threadIdx.x, pp, h)) return;
    int c[4];
    coords_of(k, par, h, c);
    const uint32_t s = (uint32_t)(c[0] + k.L[0] * (c[1] + k.L[1] * (c[2] + k.L[2] * c[3])));
    const Rng g{key0, key1, 4u * s + (uint32_t)mu, sweep};
    Su3<T> v, u, w;
    staple_sum_at<P>(v, k, gauge, c, mu);
    const int zero[4] = {0, 0, 0, 0};
    link_at<P>(u, k, gauge, c, zero, mu);
    mat_mul(w, u, v);
    const bool hb = heatbath != 0;
    subgroup<0, 1>(u, w, hb, T(beta), g, 0);
    subgroup<0, 2>(u, w, hb, T(beta), g, 1);
    subgroup<1, 2>(u, w, hb, T(beta), g, 2);
    Su3<double> ud;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) ud.m[i][j] = {(double)u.m[i][j].re, (double)u.m[i][j].im};
    // FP64: nontemporal (no thread of the launch reads a link of this direction and parity
    // but its own; 1025 -> 1007 us per heatbath sweep at 24^3 x 48)
    if constexpr (P == TMQCD_F64) LinkIO<P, TMQCD_RECON18>::template store<true>(gauge, k.gstride, par, mu, h, ud);
    else LinkIO<P, TMQCD_RECON18>::store(gauge, k.gstride, par, mu, h, ud);
}

}  // namespace

hipError_t launch_su3_sweep(const Geom& g, void* gauge, int prec, double beta, uint64_t seed, uint32_t sweep,
                            bool heatbath, hipStream_t s) {
    if (prec != TMQCD_F64 && prec != TMQCD_F32) return hipErrorInvalidValue;
    const LatK k = make_latk(g);
    const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFull), k1 = (uint32_t)(seed >> 32);
    HopParams hp{};
    hp.g = g;
    hp.prec = hp.vprec = TMQCD_F64;
    hp.nparity = 1;
    hp.nrhs = 1;
    hp.order = kOrderSlab;
    for (int mu = 0; mu < 4; ++mu)
        for (int par = 0; par < 2; ++par) {
            hp.out_parity = par;
            const stencil::HopK map = stencil::make_hopk(hp, kBlock);
            if (prec == TMQCD_F64)
                hipLaunchKernelGGL(su3_update_kernel<TMQCD_F64>, dim3(map.nblocks), dim3(kBlock), 0, s, k, map,
                                   static_cast<char*>(gauge), mu, par, beta, k0, k1, sweep, heatbath ? 1 : 0);
            else
                hipLaunchKernelGGL(su3_update_kernel<TMQCD_F32>, dim3(map.nblocks), dim3(kBlock), 0, s, k, map,
                                   static_cast<char*>(gauge), mu, par, beta, k0, k1, sweep, heatbath ? 1 : 0);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace tmqcd
