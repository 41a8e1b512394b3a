// Site coordinates, link loads and 3x3 complex products on the packed FP64
// 18-real gauge field, shared by the gauge-field kernels (HMC and heatbath).
#pragma once

#include "device.h"
#include "internal.h"

namespace tmqcd {

struct LatK {
    int L[4];
    int lxh;
    int vh;
    int nb_half;
    int64_t gstride;
};

inline LatK make_latk(const Geom& g) {
    LatK k;
    for (int i = 0; i < 4; ++i) k.L[i] = g.L[i];
    k.lxh = g.lxh;
    k.vh = (int)g.vh;
    k.nb_half = (int)((g.vh + kBlock - 1) / kBlock);
    k.gstride = g.gstride;
    return k;
}

// coordinates of the site (par, h)
__device__ __forceinline__ void coords_of(const LatK& k, int par, int h, int c[4]) {
    const int xh = h % k.lxh;
    int rest = h / k.lxh;
    c[1] = rest % k.L[1];
    rest /= k.L[1];
    c[2] = rest % k.L[2];
    c[3] = rest / k.L[2];
    c[0] = 2 * xh + ((par + c[1] + c[2] + c[3]) & 1);
}

// parity and half index of the site c + d (periodic)
__device__ __forceinline__ void site_at(const LatK& k, const int c[4], const int d[4], int& par, int& h) {
    int q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int v = c[i] + d[i];
        v = v < 0 ? v + k.L[i] : (v >= k.L[i] ? v - k.L[i] : v);
        q[i] = v;
    }
    par = (q[0] + q[1] + q[2] + q[3]) & 1;
    h = (q[0] + k.L[0] * (q[1] + k.L[1] * (q[2] + k.L[2] * q[3]))) >> 1;
}

// link U_mu at the site c + d (periodic), 18-real packed layout of storage precision P
// (FP64 by default; FP32 links load into Su3<float>)
template <int P = TMQCD_F64>
__device__ __forceinline__ void link_at(Su3<typename Prec<P>::T>& u, const LatK& k, const char* gauge, const int c[4],
                                        const int d[4], int mu) {
    int par, h;
    site_at(k, c, d, par, h);
    LinkIO<P, TMQCD_RECON18>::template load<false>(u, gauge, k.gstride, par, mu, h);
}

// a field of ncomp SU(3)-shaped matrices per site in the 18-real link layout
// (component comp of the site (par, h) at ((par * ncomp + comp) * 9 + k) * gstride + h)
__device__ __forceinline__ void mat_load(Su3<double>& u, const char* base, int64_t gstride, int ncomp, int par,
                                         int comp, int h) {
    const double2* p = reinterpret_cast<const double2*>(base) + (int64_t)((par * ncomp + comp) * 9) * gstride + h;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 w = p[k * gstride];
        u.m[k / 3][k % 3] = {w.x, w.y};
    }
}
__device__ __forceinline__ void mat_store(char* base, int64_t gstride, int ncomp, int par, int comp, int h,
                                          const Su3<double>& u) {
    double2* p = reinterpret_cast<double2*>(base) + (int64_t)((par * ncomp + comp) * 9) * gstride + h;
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k * gstride] = make_double2(u.m[k / 3][k % 3].re, u.m[k / 3][k % 3].im);
}

template <typename T>
__device__ __forceinline__ void mat_mul(Su3<T>& r, const Su3<T>& a, const Su3<T>& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[i][0] * b.m[0][j] + a.m[i][1] * b.m[1][j] + a.m[i][2] * b.m[2][j];
}
// a * b^+
template <typename T>
__device__ __forceinline__ void mat_mul_nd(Su3<T>& r, const Su3<T>& a, const Su3<T>& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.m[i][j] = cmul_cj(b.m[j][0], a.m[i][0]) + cmul_cj(b.m[j][1], a.m[i][1]) + cmul_cj(b.m[j][2], a.m[i][2]);
}
// a^+ * b
template <typename T>
__device__ __forceinline__ void mat_mul_dn(Su3<T>& r, const Su3<T>& a, const Su3<T>& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.m[i][j] = cmul_cj(a.m[0][i], b.m[0][j]) + cmul_cj(a.m[1][i], b.m[1][j]) + cmul_cj(a.m[2][i], b.m[2][j]);
}

// V_mu(x): the six Wilson staples of U_mu(x), so that the plaquettes through the
// link sum to Re Tr[U_mu(x) V_mu(x)]
template <int P = TMQCD_F64>
__device__ __forceinline__ void staple_sum_at(Su3<typename Prec<P>::T>& v, const LatK& k, const char* gauge,
                                              const int c[4], int mu) {
    using T = typename Prec<P>::T;
    const int zero[4] = {0, 0, 0, 0};
    Su3<T> a, b, t;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) v.m[i][j] = {T(0), T(0)};
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int dm[4] = {0, 0, 0, 0}, dn[4] = {0, 0, 0, 0}, dmn[4] = {0, 0, 0, 0}, dmn2[4] = {0, 0, 0, 0};
        dm[mu] = 1;
        dn[nu] = 1;
        dmn[mu] = 1;
        dmn[nu] = -1;
        dmn2[nu] = -1;
        // U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
        link_at<P>(a, k, gauge, c, dm, nu);
        link_at<P>(b, k, gauge, c, dn, mu);
        mat_mul_nd(t, a, b);
        link_at<P>(a, k, gauge, c, zero, nu);
        mat_mul_nd(b, t, a);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) v.m[i][j] = v.m[i][j] + b.m[i][j];
        // U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
        link_at<P>(a, k, gauge, c, dmn, nu);
        link_at<P>(b, k, gauge, c, dmn2, mu);
        mat_mul(t, b, a);                          // U_mu(x-nu) U_nu(x+mu-nu)
        link_at<P>(a, k, gauge, c, dmn2, nu);
        mat_mul_dn(b, t, a);                       // (U_mu U_nu)^+ U_nu(x-nu)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) v.m[i][j] = v.m[i][j] + b.m[i][j];
    }
}

}  // namespace tmqcd
