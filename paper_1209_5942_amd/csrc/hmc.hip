// Kernels of the hybrid Monte-Carlo around the solver (paper: the ensemble-
// generation section - momenta conjugate to U, the gauge force from staples,
// and the evolution U' = exp(i dt P) U):
//   * Wilson plaquette gauge force (the tree-level Symanzik action at c1 = 0),
//     G^a = (beta/3) Im Tr[T^a U_mu(x) V_mu(x)] with V_mu the six staples,
//     written or accumulated with a scale factor (momentum updates fuse here);
//   * the tree-level Symanzik force, V_mu = c0 (6 plaquette staples) + c1 (18
//     rectangle staples), c0 = 1 - 8 c1, from a stored field of plaquette
//     staples, and the rectangle sum of its action;
//   * link update U_mu(x) <- exp(i dt p^a T^a) U_mu(x): the exponential of the
//     anti-hermitian generator by a degree-16 Taylor polynomial after scaling
//     by 2^-n (||dt P|| / 2^n <= 1/4) and n squarings;
//   * deterministic two-pass reductions: the plaquette and rectangle sums, sum p^2, the
//     complex inner product of two packed FP64 spinor fields, and the change of the
//     Hamiltonian between two HMC states summed site by site (the Metropolis step's dH).
// Momenta and forces use the canonical layout double[V][4][8]; links are the
// packed FP64 18-real field, updated in place.
#include "device.h"
#include "internal.h"
#include "su3.h"
#include "stencil.h"

namespace tmqcd {
namespace {

// Im Tr(lambda^a W) for the eight Gell-Mann matrices
__device__ __forceinline__ void im_tr_lambda(const Su3<double>& q, double g[8]) {
    g[0] = q.m[1][0].im + q.m[0][1].im;
    g[1] = q.m[0][1].re - q.m[1][0].re;
    g[2] = q.m[0][0].im - q.m[1][1].im;
    g[3] = q.m[2][0].im + q.m[0][2].im;
    g[4] = q.m[0][2].re - q.m[2][0].re;
    g[5] = q.m[2][1].im + q.m[1][2].im;
    g[6] = q.m[1][2].re - q.m[2][1].re;
    g[7] = (q.m[0][0].im + q.m[1][1].im - 2.0 * q.m[2][2].im) * 0.57735026918962576451;
}

// The sites of block b for the gauge-force kernels: the hop's t-slab ranges (every
// t-slice cut into 8 ranges, range x walked slice by slice by XCD x; hardware blocks
// go round-robin over the XCDs) with the two parities interleaved, the even and the
// odd block of the same half sites in turn, so the links around a site are read by
// both parities' blocks while the XCD's L2 holds them.  Against all even blocks
// followed by all odd ones it measured, with bitwise the same forces: Wilson 144 vs
// 130 us at 16^3 x 32 and 795 vs 580 us at 24^3 x 48; tree-level Symanzik 562 vs
// 496 us and 3212 vs 2756 us.  m is the slab map of one parity (width, q, tq, slice,
// lt); the grid has 2 x 8 x lt x tq blocks.
__device__ __forceinline__ bool gauge_block_site(const stencil::HopK& m, int b, int lane, int& par, int& h) {
    const int x = b & (kNumXcd - 1), kk = b / kNumXcd;
    const int t = kk / (2 * m.tq), rem = kk - t * 2 * m.tq;
    par = rem & 1;
    const int first = x * m.q + (rem >> 1) * m.width + lane;
    const int end = min((x + 1) * m.q, m.slice);
    h = t * m.slice + first;
    return t < m.lt && first < end;
}

// one thread per site (four directions), blocks in gauge_block_site's order
__global__ __launch_bounds__(kBlock) void gauge_force_kernel(LatK k, stencil::HopK map, const char* gauge,
                                                             double* out, double coef, int accumulate) {
    int par, h;
    if (!gauge_block_site(map, blockIdx.x, threadIdx.x, par, h)) return;
    int c[4];
    coords_of(k, par, h, c);
    const int64_t s = 2 * (int64_t)h + (c[0] & 1);
    const int zero[4] = {0, 0, 0, 0};
    for (int mu = 0; mu < 4; ++mu) {
        Su3<double> v, t, u;
        staple_sum_at(v, k, gauge, c, mu);
        link_at(u, k, gauge, c, zero, mu);
        mat_mul(t, u, v);
        double g[8];
        im_tr_lambda(t, g);
        double* o = out + s * 32 + mu * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = accumulate ? o[i] + coef * g[i] : coef * g[i];
    }
}

// ------------------------------------------- tree-level Symanzik action ---
// Loops are walked as lists of signed 1-based directions: +(d+1) moves forwards
// over U_d(y), -(d+1) backwards over U_d(y - d)^+.  The rectangle R_mu_nu(x) is
// two links long in mu and one in nu: m, m, n, -m, -m, -n from x (m = mu+1,
// n = nu+1); the action's rectangle sum walks it, the force (below) builds the
// rectangle staples from stored plaquette staples.

// moves pos one step along the signed direction (selects, so pos stays in registers)
__device__ __forceinline__ void move(int pos[4], int st) {
    const int d = (st > 0 ? st : -st) - 1, delta = st > 0 ? 1 : -1;
#pragma unroll
    for (int i = 0; i < 4; ++i) pos[i] += i == d ? delta : 0;
}

// r = product of the links along `steps` from the site c + pos (pos is advanced to the end)
template <int N>
__device__ __forceinline__ void walk(Su3<double>& r, const LatK& k, const char* gauge, const int c[4], int pos[4],
                                     const int (&steps)[N]) {
    Su3<double> u, t;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int st = steps[i];
        const int d = (st > 0 ? st : -st) - 1;
        if (st < 0) move(pos, st);
        link_at(u, k, gauge, c, pos, d);
        if (st > 0) move(pos, st);
        if (i == 0) {
            if (st > 0) {
                r = u;
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) r.m[a][b] = conj(u.m[b][a]);
            }
        } else {
            if (st > 0) mat_mul(t, r, u);
            else mat_mul_nd(t, r, u);
            r = t;
        }
    }
}

__device__ __forceinline__ void add_scaled(Su3<double>& v, double c, const Su3<double>& a) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) v.m[i][j] = v.m[i][j] + scale(c, a.m[i][j]);
}

// The Symanzik force from a stored staple field.  With the single plaquette
// staples of U_mu(x),
//   Sigma+_{mu nu}(x) = U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+,
//   Sigma-_{mu nu}(x) = U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu),
// and U^+ U = 1, the three rectangle staples of side s (s = +nu or -nu) are
//   U_mu(x+mu) Sigma_s(x+mu) Sigma_s(x)          (long in mu, U_mu(x) the first link)
//   Sigma_s(x) Sigma_s(x-mu) U_mu(x-mu)          (long in mu, U_mu(x) the second link)
//   U_nu(x+mu) Sigma+(x+nu) U_nu(x)^+   or   U_nu(x+mu-nu)^+ Sigma-(x-nu) U_nu(x-nu)   (long in nu)
// so a link takes 36 products and 38 matrix loads instead of 84 products and 108
// link loads when every loop is walked.  The field holds 24 matrices per site,
// component (mu * 3 + j) * 2 + side, j the rank of nu among the directions other
// than mu, side 0 for +nu.
constexpr int kStapleComps = 24;
__device__ __forceinline__ int staple_comp(int mu, int nu, int side) {
    return (mu * 3 + (nu < mu ? nu : nu - 1)) * 2 + side;
}

// One thread per link.  The four directions of the same kBlock sites are consecutive blocks
// of one XCD (link_block: block b has direction (b / 8) % 4 and covers the sites of block
// 8 (b / 32) + b % 8 in gauge_block_site's order), so the links that the four directions'
// staples share are read while the XCD's L2 holds them; with the direction as a second grid
// dimension every direction swept the whole lattice in turn, and the Symanzik force (both of
// its kernels) took 529 instead of 492 us at 16^3 x 32 and 2794 instead of 2428 us at
// 24^3 x 48, with bitwise the same output.  This kernel stores the six staples of U_mu(x).
__device__ __forceinline__ bool link_block(const stencil::HopK& m, int b, int lane, int& mu, int& par, int& h) {
    mu = (b >> 3) & 3;
    return gauge_block_site(m, ((b >> 5) << 3) | (b & 7), lane, par, h);
}

__global__ __launch_bounds__(kBlock) void staple_field_kernel(LatK k, stencil::HopK map, const char* gauge, char* sig) {
    int mu, par, h;
    if (!link_block(map, blockIdx.x, threadIdx.x, mu, par, h)) return;
    int c[4];
    coords_of(k, par, h, c);
    const int zero[4] = {0, 0, 0, 0};
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int dm[4] = {0, 0, 0, 0}, dn[4] = {0, 0, 0, 0}, dmn[4] = {0, 0, 0, 0}, dbn[4] = {0, 0, 0, 0};
        dm[mu] = 1;
        dn[nu] = 1;
        dmn[mu] = 1;
        dmn[nu] = -1;
        dbn[nu] = -1;
        Su3<double> a, b, t;
        // + side: U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
        link_at(a, k, gauge, c, dm, nu);
        link_at(b, k, gauge, c, dn, mu);
        mat_mul_nd(t, a, b);
        link_at(a, k, gauge, c, zero, nu);
        mat_mul_nd(b, t, a);
        mat_store(sig, k.gstride, kStapleComps, par, staple_comp(mu, nu, 0), h, b);
        // - side: U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
        link_at(a, k, gauge, c, dmn, nu);
        link_at(b, k, gauge, c, dbn, mu);
        mat_mul(t, b, a);                                // U_mu(x-nu) U_nu(x+mu-nu)
        link_at(a, k, gauge, c, dbn, nu);
        mat_mul_dn(b, t, a);
        mat_store(sig, k.gstride, kStapleComps, par, staple_comp(mu, nu, 1), h, b);
    }
}

__global__ __launch_bounds__(kBlock) void gauge_force_rect_kernel(LatK k, stencil::HopK map, const char* gauge, const char* sig,
                                                                  double* out, double coef, double c0, double c1,
                                                                  int accumulate) {
    int mu, par, h;
    if (!link_block(map, blockIdx.x, threadIdx.x, mu, par, h)) return;
    int c[4];
    coords_of(k, par, h, c);
    const int zero[4] = {0, 0, 0, 0};
    int dm[4] = {0, 0, 0, 0}, dmb[4] = {0, 0, 0, 0};
    dm[mu] = 1;
    dmb[mu] = -1;
    Su3<double> v;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) v.m[i][j] = {0.0, 0.0};
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        // not unrolled: unrolling lets the compiler hoist both sides' loads (256 VGPRs and
        // AGPR spills, one wave per SIMD), which measured 20 % slower
#pragma unroll 1
        for (int side = 0; side < 2; ++side) {
            const int comp = staple_comp(mu, nu, side);
            Su3<double> sx, a, b, t;
            int pp, hh;
            mat_load(sx, sig, k.gstride, kStapleComps, par, comp, h);
            add_scaled(v, c0, sx);
            // U_mu(x+mu) Sigma(x+mu) Sigma(x)
            link_at(a, k, gauge, c, dm, mu);
            site_at(k, c, dm, pp, hh);
            mat_load(b, sig, k.gstride, kStapleComps, pp, comp, hh);
            mat_mul(t, a, b);
            mat_mul(a, t, sx);
            add_scaled(v, c1, a);
            // Sigma(x) Sigma(x-mu) U_mu(x-mu)
            site_at(k, c, dmb, pp, hh);
            mat_load(b, sig, k.gstride, kStapleComps, pp, comp, hh);
            mat_mul(t, sx, b);
            link_at(a, k, gauge, c, dmb, mu);
            mat_mul(b, t, a);
            add_scaled(v, c1, b);
            // long in nu
            int dn[4] = {0, 0, 0, 0};
            dn[nu] = side ? -1 : 1;
            site_at(k, c, dn, pp, hh);
            mat_load(b, sig, k.gstride, kStapleComps, pp, comp, hh);
            if (side == 0) {
                link_at(a, k, gauge, c, dm, nu);
                mat_mul(t, a, b);
                link_at(a, k, gauge, c, zero, nu);
                mat_mul_nd(b, t, a);
            } else {
                int dmn[4] = {0, 0, 0, 0};
                dmn[mu] = 1;
                dmn[nu] = -1;
                link_at(a, k, gauge, c, dmn, nu);
                mat_mul_dn(t, a, b);
                link_at(a, k, gauge, c, dn, nu);
                mat_mul(b, t, a);
            }
            add_scaled(v, c1, b);
        }
    }
    Su3<double> u, t;
    link_at(u, k, gauge, c, zero, mu);
    mat_mul(t, u, v);
    double g[8];
    im_tr_lambda(t, g);
    double* o = out + (2 * (int64_t)h + (c[0] & 1)) * 32 + mu * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = accumulate ? o[i] + coef * g[i] : coef * g[i];
}

// exp(A) for anti-hermitian traceless A = i dt p^a T^a: scaling, Taylor, squaring
__device__ void su3_exp_i(Su3<double>& e, const double p[8], double dt) {
    // Q = dt sum_a p^a lambda^a / 2 (hermitian); A = i Q
    const double s3 = 0.57735026918962576451;
    const double h = 0.5 * dt;
    Su3<double> a;
    // Q entries
    const C<double> q00 = {h * (p[2] + s3 * p[7]), 0.0};
    const C<double> q11 = {h * (-p[2] + s3 * p[7]), 0.0};
    const C<double> q22 = {h * (-2.0 * s3 * p[7]), 0.0};
    const C<double> q01 = {h * p[0], -h * p[1]};
    const C<double> q02 = {h * p[3], -h * p[4]};
    const C<double> q12 = {h * p[5], -h * p[6]};
    const C<double> qq[3][3] = {{q00, q01, q02}, {conj(q01), q11, q12}, {conj(q02), conj(q12), q22}};
    double nrm = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            a.m[i][j] = {-qq[i][j].im, qq[i][j].re};   // i * Q
            nrm += norm2(qq[i][j]);
        }
    nrm = sqrt(nrm);
    int n = 0;
    while (nrm > 0.25 && n < 40) {
        nrm *= 0.5;
        ++n;
    }
    const double sc = ldexp(1.0, -n);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) a.m[i][j] = scale(sc, a.m[i][j]);
    // Horner: E = I + A (I + A/2 (I + A/3 (... (I + A/16))))
    Su3<double> t;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) e.m[i][j] = {i == j ? 1.0 : 0.0, 0.0};
    for (int kk = 16; kk >= 1; --kk) {
        mat_mul(t, a, e);
        const double inv = 1.0 / kk;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) e.m[i][j] = C<double>{(i == j ? 1.0 : 0.0), 0.0} + scale(inv, t.m[i][j]);
    }
    for (int kk = 0; kk < n; ++kk) {
        mat_mul(t, e, e);
        e = t;
    }
}

__global__ __launch_bounds__(kBlock) void update_links_kernel(LatK k, char* gauge, const double* mom, double dt,
                                                              int64_t nlinks) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= nlinks) return;
    const int64_t s = idx >> 2;
    const int mu = (int)(idx & 3);
    const int x = (int)(s % k.L[0]);
    int64_t r = s / k.L[0];
    const int y = (int)(r % k.L[1]);
    r /= k.L[1];
    const int z = (int)(r % k.L[2]);
    const int t = (int)(r / k.L[2]);
    const int par = (x + y + z + t) & 1;
    double p[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) p[a] = mom[idx * 8 + a];
    Su3<double> e, u, nu;
    su3_exp_i(e, p, dt);
    LinkIO<TMQCD_F64, TMQCD_RECON18>::load<true>(u, gauge, k.gstride, par, mu, s >> 1);
    mat_mul(nu, e, u);
    LinkIO<TMQCD_F64, TMQCD_RECON18>::store(gauge, k.gstride, par, mu, s >> 1, nu);
}

// ----------------------------------------------------------- reductions ---
template <int N>
__global__ __launch_bounds__(kBlock) void finalize_kernel(const double* partials, int nblocks, double* result) {
    double tot[N];
    sum_partials<N>(partials, nblocks, tot);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) result[i] = tot[i];
}

// sum over the site's 6 plaquettes P_mu_nu(x), mu < nu, of Re Tr
__device__ double plaquette_site(const LatK& k, const char* gauge, const int c[4]) {
    const int zero[4] = {0, 0, 0, 0};
    double v = 0.0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) {
            int dm[4] = {0, 0, 0, 0}, dn[4] = {0, 0, 0, 0};
            dm[mu] = 1;
            dn[nu] = 1;
            Su3<double> a, b, t1, t2;
            link_at(a, k, gauge, c, zero, mu);
            link_at(b, k, gauge, c, dm, nu);
            mat_mul(t1, a, b);                     // U_mu(x) U_nu(x+mu)
            link_at(a, k, gauge, c, zero, nu);
            link_at(b, k, gauge, c, dn, mu);
            mat_mul(t2, a, b);                     // U_nu(x) U_mu(x+nu)
            // Re Tr[t1 t2^+]
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) v += t1.m[i][j].re * t2.m[i][j].re + t1.m[i][j].im * t2.m[i][j].im;
        }
    return v;
}

// sum over the site's 12 rectangles R_mu_nu(x), mu != nu, of Re Tr
__device__ double rectangle_site(const LatK& k, const char* gauge, const int c[4]) {
    double v = 0.0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu) {
            if (nu == mu) continue;
            const int m = mu + 1, n = nu + 1;
            int pos[4] = {0, 0, 0, 0};
            const int st[6] = {m, m, n, -m, -m, -n};
            Su3<double> r;
            walk(r, k, gauge, c, pos, st);
            v += r.m[0][0].re + r.m[1][1].re + r.m[2][2].re;
        }
    return v;
}

__global__ __launch_bounds__(kBlock) void plaquette_kernel(LatK k, const char* gauge, double* partials) {
    const int par = blockIdx.x >= (unsigned)k.nb_half ? 1 : 0;
    const int h = (blockIdx.x - par * k.nb_half) * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (h < k.vh) {
        int c[4];
        coords_of(k, par, h, c);
        v[0] = plaquette_site(k, gauge, c);
    }
    block_partial<1>(v, partials, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void rectangle_kernel(LatK k, const char* gauge, double* partials) {
    const int par = blockIdx.x >= (unsigned)k.nb_half ? 1 : 0;
    const int h = (blockIdx.x - par * k.nb_half) * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (h < k.vh) {
        int c[4];
        coords_of(k, par, h, c);
        v[0] = rectangle_site(k, gauge, c);
    }
    block_partial<1>(v, partials, blockIdx.x);
}

// The change of the HMC Hamiltonian between two states, accumulated site by site
// in FP64 (no difference of two large totals): per site x
//   kinetic   1/2 sum_{mu,a} (p1^2 - p0^2)
//   gauge     (beta/3) [c0 sum_{mu<nu} Re Tr(P0 - P1) + c1 sum_{mu!=nu} Re Tr(R0 - R1)]
//   fermion   Re phi(x)^+ (X1(x) - X0(x))      (sites of the pseudofermion's subset)
// and their sum; block sums of (total, kinetic, gauge, fermion), finished by a
// second launch in a fixed order.
struct DeltaHK {
    LatK k;
    const char *u0, *u1;
    const double *p0, *p1;
    const char *phi, *x0, *x1;
    int64_t stride, hbytes;
    double beta, c0, c1;
    int fermion_parities;   // 1: even sites only (the even-odd action), 2: all
};

__global__ __launch_bounds__(kBlock) void delta_h_kernel(DeltaHK a, double* partials) {
    const LatK& k = a.k;
    const int par = blockIdx.x >= (unsigned)k.nb_half ? 1 : 0;
    const int h = (blockIdx.x - par * k.nb_half) * kBlock + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (h < k.vh) {
        int c[4];
        coords_of(k, par, h, c);
        const int64_t s = 2 * (int64_t)h + (c[0] & 1);
        double kin = 0.0;
        for (int i = 0; i < 32; ++i) {
            const double q1 = a.p1[s * 32 + i], q0 = a.p0[s * 32 + i];
            kin += 0.5 * (q1 - q0) * (q1 + q0);
        }
        double gauge = 0.0;
        if (a.beta != 0.0) {
            gauge = a.c0 * (plaquette_site(k, a.u0, c) - plaquette_site(k, a.u1, c));
            if (a.c1 != 0.0) gauge += a.c1 * (rectangle_site(k, a.u0, c) - rectangle_site(k, a.u1, c));
            gauge *= a.beta / 3.0;
        }
        double ferm = 0.0;
        if (par < a.fermion_parities) {
            const int64_t off = par * a.hbytes;
            Spinor<double> f, y0, y1;
            SpinorIO<TMQCD_F64>::load(f, a.phi + off, a.stride, h);
            SpinorIO<TMQCD_F64>::load(y0, a.x0 + off, a.stride, h);
            SpinorIO<TMQCD_F64>::load(y1, a.x1 + off, a.stride, h);
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) ferm += cmul_cj(f.s[sp][cc], y1.s[sp][cc] - y0.s[sp][cc]).re;
        }
        v[0] = kin + gauge + ferm;
        v[1] = kin;
        v[2] = gauge;
        v[3] = ferm;
    }
    block_partial<4>(v, partials, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void mom_norm2_kernel(const double* mom, int64_t n, double* partials) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (i < n) {
#pragma unroll
        for (int a = 0; a < 8; ++a) v[0] += mom[i * 8 + a] * mom[i * 8 + a];
    }
    block_partial<1>(v, partials, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void spinor_dot_kernel(const char* x, const char* y, int64_t stride, int vh,
                                                            int nhalf, int64_t hbytes, double* partials) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (i < nhalf * vh) {
        const int half = i / vh, h = i - half * vh;
        Spinor<double> a, b;
        SpinorIO<TMQCD_F64>::load(a, x + half * hbytes, stride, h);
        SpinorIO<TMQCD_F64>::load(b, y + half * hbytes, stride, h);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const C<double> z = cmul_cj(a.s[s][c], b.s[s][c]);
                v[0] += z.re;
                v[1] += z.im;
            }
    }
    block_partial<2>(v, partials, blockIdx.x);
}

}  // namespace

int64_t aux_partials_doubles(const Geom& g) {
    // the largest among the reductions: the momentum norm (8 V_h threads, one value per block) and the
    // Hamiltonian difference (2 V_h threads, four values per block)
    const int64_t mom = (8 * g.vh + kBlock - 1) / kBlock, dh = 4 * 2 * ((g.vh + kBlock - 1) / kBlock);
    return 2 * (mom > dh ? mom : dh) + 4;
}

hipError_t launch_gauge_force(const Geom& g, const void* gauge, double beta, double* out, double scale, int accumulate,
                              hipStream_t s) {
    const LatK k = make_latk(g);
    HopParams hp{};
    hp.g = g;
    hp.prec = hp.vprec = TMQCD_F64;
    hp.nparity = 2;
    hp.nrhs = 1;
    hp.order = kOrderSlab;
    const stencil::HopK map = stencil::make_hopk(hp, kBlock);
    // G^a = (beta/3) Im Tr[T^a U V] = (beta/6) Im Tr[lambda^a U V]
    hipLaunchKernelGGL(gauge_force_kernel, dim3(map.nblocks), dim3(kBlock), 0, s, k, map,
                       static_cast<const char*>(gauge), out, scale * beta / 6.0, accumulate);
    return hipGetLastError();
}

int64_t staple_field_bytes(const Geom& g) { return (int64_t)2 * kStapleComps * 9 * 16 * g.gstride; }

hipError_t launch_gauge_force_sym(const Geom& g, const void* gauge, double beta, double c1, double* out, double scale,
                                  int accumulate, void* ws, hipStream_t s) {
    const LatK k = make_latk(g);
    const double coef = scale * beta / 6.0;
    HopParams hp{};
    hp.g = g;
    hp.prec = hp.vprec = TMQCD_F64;
    hp.nparity = 2;
    hp.nrhs = 1;
    hp.order = kOrderSlab;
    const stencil::HopK map = stencil::make_hopk(hp, kBlock);
    if (c1 == 0.0) {   // the Wilson action: plaquette staples only
        hipLaunchKernelGGL(gauge_force_kernel, dim3(map.nblocks), dim3(kBlock), 0, s, k, map,
                           static_cast<const char*>(gauge), out, coef, accumulate);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(staple_field_kernel, dim3(4 * map.nblocks), dim3(kBlock), 0, s, k, map,
                       static_cast<const char*>(gauge), static_cast<char*>(ws));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gauge_force_rect_kernel, dim3(4 * map.nblocks), dim3(kBlock), 0, s, k, map,
                       static_cast<const char*>(gauge), static_cast<const char*>(ws), out, coef, 1.0 - 8.0 * c1, c1,
                       accumulate);
    return hipGetLastError();
}

hipError_t launch_rectangle(const Geom& g, const void* gauge, double* result, double* partials, hipStream_t s) {
    const LatK k = make_latk(g);
    const int nb = 2 * k.nb_half;
    hipLaunchKernelGGL(rectangle_kernel, dim3(nb), dim3(kBlock), 0, s, k, static_cast<const char*>(gauge), partials);
    hipLaunchKernelGGL((finalize_kernel<1>), dim3(1), dim3(kBlock), 0, s, partials, nb, result);
    return hipGetLastError();
}

hipError_t launch_update_links(const Geom& g, void* gauge, const double* mom, double dt, hipStream_t s) {
    const LatK k = make_latk(g);
    const int64_t n = 8 * g.vh;
    hipLaunchKernelGGL(update_links_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, k,
                       static_cast<char*>(gauge), mom, dt, n);
    return hipGetLastError();
}

hipError_t launch_plaquette(const Geom& g, const void* gauge, double* result, double* partials, hipStream_t s) {
    const LatK k = make_latk(g);
    const int nb = 2 * k.nb_half;
    hipLaunchKernelGGL(plaquette_kernel, dim3(nb), dim3(kBlock), 0, s, k, static_cast<const char*>(gauge), partials);
    hipLaunchKernelGGL((finalize_kernel<1>), dim3(1), dim3(kBlock), 0, s, partials, nb, result);
    return hipGetLastError();
}

hipError_t launch_mom_norm2(const Geom& g, const double* mom, double* result, double* partials, hipStream_t s) {
    const int64_t n = 8 * g.vh;
    const int nb = (int)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(mom_norm2_kernel, dim3(nb), dim3(kBlock), 0, s, mom, n, partials);
    hipLaunchKernelGGL((finalize_kernel<1>), dim3(1), dim3(kBlock), 0, s, partials, nb, result);
    return hipGetLastError();
}

hipError_t launch_delta_h(const Geom& g, const void* u0, const void* u1, const double* p0, const double* p1,
                          const void* phi, const void* x0, const void* x1, int fermion_parities, double beta, double c1,
                          double* result, double* partials, hipStream_t s) {
    DeltaHK a;
    a.k = make_latk(g);
    a.u0 = static_cast<const char*>(u0);
    a.u1 = static_cast<const char*>(u1);
    a.p0 = p0;
    a.p1 = p1;
    a.phi = static_cast<const char*>(phi);
    a.x0 = static_cast<const char*>(x0);
    a.x1 = static_cast<const char*>(x1);
    a.stride = g.stride;
    a.hbytes = half_field_bytes(g, TMQCD_F64);
    a.beta = beta;
    a.c0 = 1.0 - 8.0 * c1;
    a.c1 = c1;
    a.fermion_parities = fermion_parities;
    const int nb = 2 * a.k.nb_half;
    hipLaunchKernelGGL(delta_h_kernel, dim3(nb), dim3(kBlock), 0, s, a, partials);
    hipLaunchKernelGGL((finalize_kernel<4>), dim3(1), dim3(kBlock), 0, s, partials, nb, result);
    return hipGetLastError();
}

hipError_t launch_spinor_dot(const Geom& g, const void* x, const void* y, int nhalf, double* result, double* partials,
                             hipStream_t s) {
    const int nb = (int)((nhalf * g.vh + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(spinor_dot_kernel, dim3(nb), dim3(kBlock), 0, s, static_cast<const char*>(x),
                       static_cast<const char*>(y), g.stride, (int)g.vh, nhalf, half_field_bytes(g, TMQCD_F64),
                       partials);
    hipLaunchKernelGGL((finalize_kernel<2>), dim3(1), dim3(kBlock), 0, s, partials, nb, result);
    return hipGetLastError();
}

}  // namespace tmqcd
