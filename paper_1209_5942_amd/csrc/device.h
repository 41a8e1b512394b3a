// Device-side types: complex arithmetic, spinor and SU(3) registers, per-precision
// site loads/stores of the packed layouts, wavefront reductions.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "layout.h"

namespace tmqcd {

// ---------------------------------------------------------------- complex ---
template <typename T>
struct C {
    T re, im;
};
template <typename T>
__device__ __forceinline__ C<T> operator+(C<T> a, C<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ C<T> operator-(C<T> a, C<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ C<T> operator*(C<T> a, C<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ C<T> scale(T s, C<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__device__ __forceinline__ C<T> conj(C<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T>
__device__ __forceinline__ C<T> cmul_cj(C<T> a, C<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ T norm2(C<T> a) { return a.re * a.re + a.im * a.im; }
// multiply by the phase i^code: 0 -> 1, 1 -> i, 2 -> -1, 3 -> -i
template <int CODE, typename T>
__device__ __forceinline__ C<T> mul_i(C<T> z) {
    constexpr int c = CODE & 3;
    if constexpr (c == 0) return z;
    else if constexpr (c == 1) return {-z.im, z.re};
    else if constexpr (c == 2) return {-z.re, -z.im};
    else return {z.im, -z.re};
}
template <typename T>
__device__ __forceinline__ C<T> cvt(C<double> z) { return {(T)z.re, (T)z.im}; }

template <typename T>
struct Spinor {
    C<T> s[4][3];   // [spin][colour]
};
template <typename T>
struct Half {
    C<T> s[2][3];
};
template <typename T>
struct Su3 {
    C<T> m[3][3];
};

// ----------------------------------------------------- precision traits ---
template <int P>
struct Prec {
    using T = float;   // FP32 and FP16 storage compute in FP32
};
template <>
struct Prec<TMQCD_F64> {
    using T = double;
};

// ------------------------------------------------------- streaming access ---
// Links are read exactly once per hop; nontemporal loads keep them from
// displacing the neighbour spinors that other sites will read again.
template <typename V>
__device__ __forceinline__ V ld_stream(const V* p) {
    if constexpr (sizeof(V) == 16) {
        typedef int v4 __attribute__((ext_vector_type(4)));
        return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const v4*>(p)));
    } else if constexpr (sizeof(V) == 8) {
        typedef int v2 __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const v2*>(p)));
    } else {
        static_assert(sizeof(V) == 4, "unsupported link unit");
        return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const int*>(p)));
    }
}

// Nontemporal store: results written once and not read again by the launch
// (the multi-RHS outputs) stay out of the way of the spinors it still reads.
template <typename V>
__device__ __forceinline__ void st_stream(V* p, const V& v) {
    static_assert(sizeof(V) == 16, "16-byte units");
    typedef int v4 __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(__builtin_bit_cast(v4, v), reinterpret_cast<v4*>(p));
}

// ------------------------------------------------------- spinor site I/O ---
// `base` points at one packed half field; `stride` is its SoA stride.
template <int P>
struct SpinorIO;

template <>
struct SpinorIO<TMQCD_F64> {
    using T = double;
    __device__ __forceinline__ static void load(Spinor<T>& v, const char* base, int64_t stride, int64_t h) {
        const double2* p = reinterpret_cast<const double2*>(base) + h;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            double2 w = p[k * stride];
            v.s[k / 3][k % 3] = {w.x, w.y};
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ static void store(char* base, int64_t stride, int64_t h, const Spinor<T>& v) {
        double2* p = reinterpret_cast<double2*>(base) + h;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double2 w = make_double2(v.s[k / 3][k % 3].re, v.s[k / 3][k % 3].im);
            if constexpr (NT) st_stream(p + k * stride, w);
            else p[k * stride] = w;
        }
    }
};

template <>
struct SpinorIO<TMQCD_F32> {
    using T = float;
    __device__ __forceinline__ static void load(Spinor<T>& v, const char* base, int64_t stride, int64_t h) {
        const float4* p = reinterpret_cast<const float4*>(base) + h;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float4 w = p[k * stride];
            v.s[(2 * k) / 3][(2 * k) % 3] = {w.x, w.y};
            v.s[(2 * k + 1) / 3][(2 * k + 1) % 3] = {w.z, w.w};
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ static void store(char* base, int64_t stride, int64_t h, const Spinor<T>& v) {
        float4* p = reinterpret_cast<float4*>(base) + h;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const C<T> a = v.s[(2 * k) / 3][(2 * k) % 3], b = v.s[(2 * k + 1) / 3][(2 * k + 1) % 3];
            const float4 w = make_float4(a.re, a.im, b.re, b.im);
            if constexpr (NT) st_stream(p + k * stride, w);
            else p[k * stride] = w;
        }
    }
};

// FP16: 24 halves in three 16-byte units, scaled by a per-site FP32 factor equal
// to the largest |component|; a site whose components are all zero stores zeros.
template <>
struct SpinorIO<TMQCD_F16> {
    using T = float;
    union U16 {
        uint4 u;
        __half h[8];
    };
    __device__ __forceinline__ static void load(Spinor<T>& v, const char* base, int64_t stride, int64_t h) {
        const uint4* p = reinterpret_cast<const uint4*>(base) + h;
        const float s = reinterpret_cast<const float*>(base + 48 * stride)[h];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            U16 w;
            w.u = p[k * stride];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * k + j;
                v.s[c / 3][c % 3] = {s * __half2float(w.h[2 * j]), s * __half2float(w.h[2 * j + 1])};
            }
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ static void store(char* base, int64_t stride, int64_t h, const Spinor<T>& v) {
        float m = 0.f;
#pragma unroll
        for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v.s[c / 3][c % 3].re), fabsf(v.s[c / 3][c % 3].im)));
        const float inv = m > 0.f ? 1.f / m : 0.f;
        uint4* p = reinterpret_cast<uint4*>(base) + h;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            U16 w;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * k + j;
                w.h[2 * j] = __float2half_rn(v.s[c / 3][c % 3].re * inv);
                w.h[2 * j + 1] = __float2half_rn(v.s[c / 3][c % 3].im * inv);
            }
            if constexpr (NT) st_stream(p + k * stride, w.u);
            else p[k * stride] = w.u;
        }
        reinterpret_cast<float*>(base + 48 * stride)[h] = m;
    }
};

// --------------------------------------------------------- link site I/O ---

// `base` points at the whole packed gauge field; the link of direction mu whose
// origin site has parity `par` and half index h.
template <typename T>
__device__ __forceinline__ void rebuild_third_row(Su3<T>& u) {
    // row 2 = conj(row 0 x row 1), exact for unitary U with det U = 1
    u.m[2][0] = conj(u.m[0][1] * u.m[1][2] - u.m[0][2] * u.m[1][1]);
    u.m[2][1] = conj(u.m[0][2] * u.m[1][0] - u.m[0][0] * u.m[1][2]);
    u.m[2][2] = conj(u.m[0][0] * u.m[1][1] - u.m[0][1] * u.m[1][0]);
}

template <int P, int R>
struct LinkIO;

template <int R>
struct LinkIO64 {
    static_assert(R == TMQCD_RECON18 || R == TMQCD_RECON12, "18- or 12-real FP64 links");
    using T = double;
    using Unit = double2;
    static constexpr int kUnits = R == TMQCD_RECON18 ? 9 : 6;
    // STREAM: nontemporal loads (the link is read once); false where links are re-read
    template <bool STREAM = true>
    __device__ __forceinline__ static void load(Su3<T>& u, const char* base, int64_t gstride, int par, int mu,
                                                int64_t h) {
        const double2* p = reinterpret_cast<const double2*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
#pragma unroll
        for (int k = 0; k < kUnits; ++k) {
            const double2 w = STREAM ? ld_stream(p + k * gstride) : p[k * gstride];
            u.m[k / 3][k % 3] = {w.x, w.y};
        }
        if constexpr (R == TMQCD_RECON12) rebuild_third_row(u);
    }
    // NT: nontemporal stores, for links the launch does not read back
    template <bool NT = false>
    __device__ __forceinline__ static void store(char* base, int64_t gstride, int par, int mu, int64_t h,
                                                 const Su3<double>& u) {
        double2* p = reinterpret_cast<double2*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
#pragma unroll
        for (int k = 0; k < kUnits; ++k) {
            const double2 w = make_double2(u.m[k / 3][k % 3].re, u.m[k / 3][k % 3].im);
            if constexpr (NT) st_stream(p + k * gstride, w);
            else p[k * gstride] = w;
        }
    }
};
template <>
struct LinkIO<TMQCD_F64, TMQCD_RECON18> : LinkIO64<TMQCD_RECON18> {};
template <>
struct LinkIO<TMQCD_F64, TMQCD_RECON12> : LinkIO64<TMQCD_RECON12> {};

template <>
struct LinkIO<TMQCD_F32, TMQCD_RECON18> {
    using T = float;
    using Unit = float2;
    static constexpr int kUnits = 9;
    template <bool STREAM = true>
    __device__ __forceinline__ static void load(Su3<T>& u, const char* base, int64_t gstride, int par, int mu,
                                                int64_t h) {
        const float2* p = reinterpret_cast<const float2*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float2 w = STREAM ? ld_stream(p + k * gstride) : p[k * gstride];
            u.m[k / 3][k % 3] = {w.x, w.y};
        }
    }
    __device__ __forceinline__ static void store(char* base, int64_t gstride, int par, int mu, int64_t h,
                                                 const Su3<double>& u) {
        float2* p = reinterpret_cast<float2*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
#pragma unroll
        for (int k = 0; k < 9; ++k) p[k * gstride] = make_float2((float)u.m[k / 3][k % 3].re, (float)u.m[k / 3][k % 3].im);
    }
};

template <>
struct LinkIO<TMQCD_F32, TMQCD_RECON12> {
    using T = float;
    using Unit = float4;
    static constexpr int kUnits = 3;
    template <bool STREAM = true>
    __device__ __forceinline__ static void load(Su3<T>& u, const char* base, int64_t gstride, int par, int mu,
                                                int64_t h) {
        const float4* p = reinterpret_cast<const float4*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float4 w = STREAM ? ld_stream(p + k * gstride) : p[k * gstride];
            u.m[(2 * k) / 3][(2 * k) % 3] = {w.x, w.y};
            u.m[(2 * k + 1) / 3][(2 * k + 1) % 3] = {w.z, w.w};
        }
        rebuild_third_row(u);
    }
    __device__ __forceinline__ static void store(char* base, int64_t gstride, int par, int mu, int64_t h,
                                                 const Su3<double>& u) {
        float4* p = reinterpret_cast<float4*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const C<double> a = u.m[(2 * k) / 3][(2 * k) % 3], b = u.m[(2 * k + 1) / 3][(2 * k + 1) % 3];
            p[k * gstride] = make_float4((float)a.re, (float)a.im, (float)b.re, (float)b.im);
        }
    }
};

template <>
struct LinkIO<TMQCD_F16, TMQCD_RECON18> {
    using T = float;
    using Unit = __half2;
    static constexpr int kUnits = 9;
    template <bool STREAM = true>
    __device__ __forceinline__ static void load(Su3<T>& u, const char* base, int64_t gstride, int par, int mu,
                                                int64_t h) {
        const __half2* p = reinterpret_cast<const __half2*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float2 w = __half22float2(STREAM ? ld_stream(p + k * gstride) : p[k * gstride]);
            u.m[k / 3][k % 3] = {w.x, w.y};
        }
    }
    __device__ __forceinline__ static void store(char* base, int64_t gstride, int par, int mu, int64_t h,
                                                 const Su3<double>& u) {
        __half2* p = reinterpret_cast<__half2*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
#pragma unroll
        for (int k = 0; k < 9; ++k)
            p[k * gstride] = __halves2half2(__float2half_rn((float)u.m[k / 3][k % 3].re),
                                            __float2half_rn((float)u.m[k / 3][k % 3].im));
    }
};

template <>
struct LinkIO<TMQCD_F16, TMQCD_RECON12> {
    using T = float;
    using Unit = uint2;
    static constexpr int kUnits = 3;
    union U8 {
        uint2 u;
        __half h[4];
    };
    template <bool STREAM = true>
    __device__ __forceinline__ static void load(Su3<T>& u, const char* base, int64_t gstride, int par, int mu,
                                                int64_t h) {
        const uint2* p = reinterpret_cast<const uint2*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            U8 w;
            w.u = STREAM ? ld_stream(p + k * gstride) : p[k * gstride];
            u.m[(2 * k) / 3][(2 * k) % 3] = {__half2float(w.h[0]), __half2float(w.h[1])};
            u.m[(2 * k + 1) / 3][(2 * k + 1) % 3] = {__half2float(w.h[2]), __half2float(w.h[3])};
        }
        rebuild_third_row(u);
    }
    __device__ __forceinline__ static void store(char* base, int64_t gstride, int par, int mu, int64_t h,
                                                 const Su3<double>& u) {
        uint2* p = reinterpret_cast<uint2*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const C<double> a = u.m[(2 * k) / 3][(2 * k) % 3], b = u.m[(2 * k + 1) / 3][(2 * k + 1) % 3];
            U8 w;
            w.h[0] = __float2half_rn((float)a.re);
            w.h[1] = __float2half_rn((float)a.im);
            w.h[2] = __float2half_rn((float)b.re);
            w.h[3] = __float2half_rn((float)b.im);
            p[k * gstride] = w.u;
        }
    }
};

// ------------------------------------------------- REC10 and REC8 links ---
// REC10 keeps the first row a and the first column (a1, b1, c1); b2, b3 solve
// conj(a2) b2 + conj(a3) b3 = -conj(a1) b1 (b orthogonal to a) and
// -a3 b2 + a2 b3 = conj(c1) (the first entry of c = conj(a x b)), and
// c2, c3 follow from c = conj(a x b); written out with n = 1/(|a2|^2 + |a3|^2):
template <typename T>
__device__ __forceinline__ void complete_from_row_col(Su3<T>& u) {
    const C<T> a1 = u.m[0][0], a2 = u.m[0][1], a3 = u.m[0][2], b1 = u.m[1][0], c1 = u.m[2][0];
    const T n = T(1) / (norm2(a2) + norm2(a3));
    const C<T> a1c = conj(a1), c1c = conj(c1), b1c = conj(b1);
    u.m[1][1] = scale(-n, b1 * a1c * a2 + c1c * conj(a3));
    u.m[1][2] = scale(-n, b1 * a1c * a3 - c1c * conj(a2));
    u.m[2][1] = scale(n, b1c * conj(a3) - c1 * a1c * a2);
    u.m[2][2] = scale(-n, b1c * conj(a2) + c1 * a1c * a3);
}

__device__ __forceinline__ void sincos_pi(double x, double* s, double* c) { sincospi(x, s, c); }
__device__ __forceinline__ void sincos_pi(float x, float* s, float* c) { sincospif(x, s, c); }

// REC8: a1 and c1 from their phases (stored as angle / pi) and the unit norms of
// the first row and the first column, then as REC10
template <typename T>
__device__ __forceinline__ void complete_rec8(Su3<T>& u, T tha, T thc) {
    const T ra = sqrt(fmax(T(0), T(1) - norm2(u.m[0][1]) - norm2(u.m[0][2])));
    T s, c;
    sincos_pi(tha, &s, &c);
    u.m[0][0] = {ra * c, ra * s};
    const T rc = sqrt(fmax(T(0), T(1) - ra * ra - norm2(u.m[1][0])));
    sincos_pi(thc, &s, &c);
    u.m[2][0] = {rc * c, rc * s};
    complete_from_row_col(u);
}
__host__ __device__ inline double phase_over_pi(const C<double>& z) { return atan2(z.im, z.re) / M_PI; }

// one complex entry per unit: FP64 double2, FP32 float2, FP16 half2
template <int P>
struct Entry;
template <>
struct Entry<TMQCD_F64> {
    using T = double;
    using Unit = double2;
    __device__ __forceinline__ static C<T> get(Unit w) { return {w.x, w.y}; }
    __device__ __forceinline__ static Unit put(const C<double>& z) { return make_double2(z.re, z.im); }
};
template <>
struct Entry<TMQCD_F32> {
    using T = float;
    using Unit = float2;
    __device__ __forceinline__ static C<T> get(Unit w) { return {w.x, w.y}; }
    __device__ __forceinline__ static Unit put(const C<double>& z) { return make_float2((float)z.re, (float)z.im); }
};
template <>
struct Entry<TMQCD_F16> {
    using T = float;
    using Unit = __half2;
    __device__ __forceinline__ static C<T> get(Unit w) {
        const float2 f = __half22float2(w);
        return {f.x, f.y};
    }
    __device__ __forceinline__ static Unit put(const C<double>& z) {
        return __halves2half2(__float2half_rn((float)z.re), __float2half_rn((float)z.im));
    }
};

// REC10: units a1, a2, a3, b1, c1
template <int P>
struct LinkIO10 {
    using E = Entry<P>;
    using T = typename E::T;
    using Unit = typename E::Unit;
    static constexpr int kUnits = 5;
    template <bool STREAM = true>
    __device__ __forceinline__ static void load(Su3<T>& u, const char* base, int64_t gstride, int par, int mu,
                                                int64_t h) {
        const Unit* p = reinterpret_cast<const Unit*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
        C<T> e[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) e[k] = E::get(STREAM ? ld_stream(p + k * gstride) : p[k * gstride]);
        u.m[0][0] = e[0];
        u.m[0][1] = e[1];
        u.m[0][2] = e[2];
        u.m[1][0] = e[3];
        u.m[2][0] = e[4];
        complete_from_row_col(u);
    }
    __device__ __forceinline__ static void store(char* base, int64_t gstride, int par, int mu, int64_t h,
                                                 const Su3<double>& u) {
        Unit* p = reinterpret_cast<Unit*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
        p[0] = E::put(u.m[0][0]);
        p[gstride] = E::put(u.m[0][1]);
        p[2 * gstride] = E::put(u.m[0][2]);
        p[3 * gstride] = E::put(u.m[1][0]);
        p[4 * gstride] = E::put(u.m[2][0]);
    }
};
template <>
struct LinkIO<TMQCD_F64, TMQCD_RECON10> : LinkIO10<TMQCD_F64> {};
template <>
struct LinkIO<TMQCD_F32, TMQCD_RECON10> : LinkIO10<TMQCD_F32> {};
template <>
struct LinkIO<TMQCD_F16, TMQCD_RECON10> : LinkIO10<TMQCD_F16> {};

// REC8, FP64: units (theta_a / pi, theta_c / pi), a2, a3, b1
template <>
struct LinkIO<TMQCD_F64, TMQCD_RECON8> {
    using T = double;
    using Unit = double2;
    static constexpr int kUnits = 4;
    template <bool STREAM = true>
    __device__ __forceinline__ static void load(Su3<T>& u, const char* base, int64_t gstride, int par, int mu,
                                                int64_t h) {
        const double2* p = reinterpret_cast<const double2*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
        double2 w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = STREAM ? ld_stream(p + k * gstride) : p[k * gstride];
        u.m[0][1] = {w[1].x, w[1].y};
        u.m[0][2] = {w[2].x, w[2].y};
        u.m[1][0] = {w[3].x, w[3].y};
        complete_rec8(u, w[0].x, w[0].y);
    }
    __device__ __forceinline__ static void store(char* base, int64_t gstride, int par, int mu, int64_t h,
                                                 const Su3<double>& u) {
        double2* p = reinterpret_cast<double2*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
        p[0] = make_double2(phase_over_pi(u.m[0][0]), phase_over_pi(u.m[2][0]));
        p[gstride] = make_double2(u.m[0][1].re, u.m[0][1].im);
        p[2 * gstride] = make_double2(u.m[0][2].re, u.m[0][2].im);
        p[3 * gstride] = make_double2(u.m[1][0].re, u.m[1][0].im);
    }
};

// REC8, FP32: units (theta_a / pi, theta_c / pi, a2), (a3, b1)
template <>
struct LinkIO<TMQCD_F32, TMQCD_RECON8> {
    using T = float;
    using Unit = float4;
    static constexpr int kUnits = 2;
    template <bool STREAM = true>
    __device__ __forceinline__ static void load(Su3<T>& u, const char* base, int64_t gstride, int par, int mu,
                                                int64_t h) {
        const float4* p = reinterpret_cast<const float4*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
        const float4 w0 = STREAM ? ld_stream(p) : p[0];
        const float4 w1 = STREAM ? ld_stream(p + gstride) : p[gstride];
        u.m[0][1] = {w0.z, w0.w};
        u.m[0][2] = {w1.x, w1.y};
        u.m[1][0] = {w1.z, w1.w};
        complete_rec8(u, w0.x, w0.y);
    }
    __device__ __forceinline__ static void store(char* base, int64_t gstride, int par, int mu, int64_t h,
                                                 const Su3<double>& u) {
        float4* p = reinterpret_cast<float4*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
        p[0] = make_float4((float)phase_over_pi(u.m[0][0]), (float)phase_over_pi(u.m[2][0]), (float)u.m[0][1].re,
                           (float)u.m[0][1].im);
        p[gstride] = make_float4((float)u.m[0][2].re, (float)u.m[0][2].im, (float)u.m[1][0].re, (float)u.m[1][0].im);
    }
};

// REC8, FP16: one unit of eight halves (theta_a / pi, theta_c / pi, a2, a3, b1)
template <>
struct LinkIO<TMQCD_F16, TMQCD_RECON8> {
    using T = float;
    using Unit = uint4;
    static constexpr int kUnits = 1;
    union U16 {
        uint4 u;
        __half h[8];
    };
    template <bool STREAM = true>
    __device__ __forceinline__ static void load(Su3<T>& u, const char* base, int64_t gstride, int par, int mu,
                                                int64_t h) {
        const uint4* p = reinterpret_cast<const uint4*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
        U16 w;
        w.u = STREAM ? ld_stream(p) : p[0];
        u.m[0][1] = {__half2float(w.h[2]), __half2float(w.h[3])};
        u.m[0][2] = {__half2float(w.h[4]), __half2float(w.h[5])};
        u.m[1][0] = {__half2float(w.h[6]), __half2float(w.h[7])};
        complete_rec8(u, __half2float(w.h[0]), __half2float(w.h[1]));
    }
    __device__ __forceinline__ static void store(char* base, int64_t gstride, int par, int mu, int64_t h,
                                                 const Su3<double>& u) {
        uint4* p = reinterpret_cast<uint4*>(base) + (int64_t)((par * 4 + mu) * kUnits) * gstride + h;
        U16 w;
        const double v[8] = {phase_over_pi(u.m[0][0]), phase_over_pi(u.m[2][0]), u.m[0][1].re, u.m[0][1].im,
                             u.m[0][2].re, u.m[0][2].im, u.m[1][0].re, u.m[1][0].im};
#pragma unroll
        for (int k = 0; k < 8; ++k) w.h[k] = __float2half_rn((float)v[k]);
        p[0] = w.u;
    }
};

// ------------------------------------------------------------ scheduling ---
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Remap so that XCD k works on one contiguous range of logical blocks: the
// neighbour spinors a block reads are then mostly those its XCD read recently.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_swizzle(int bid, int nblocks) {
    const int q = nblocks / kNumXcd, rem = nblocks % kNumXcd;
    const int k = bid % kNumXcd, j = bid / kNumXcd;
    return k * q + (k < rem ? k : rem) + j;
}

// ------------------------------------------------------------ reductions ---
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMinBlock = 128;   // smallest block of a tunable hop launch (sizes the partial sums)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Solver scalars, resident in device memory so that a queue of iterations runs
// without host round trips.
struct CgState {
    double rr;        // |r|^2 of the current residual
    double rr_prev;   // |r|^2 before the last update
    double pAp;       // p^+ A p
    double alpha, beta;
    double stop_rr;   // the update kernel flags done when rr <= stop_rr
    int iter;         // iterations completed
    int max_iter;
    int cycle_end;    // the update kernel flags done when iter reaches it (reliable-update cycle cap)
    int done;         // 0 running, 1 reached stop_rr or cycle_end, 2 breakdown, 3 iteration cap
    int beta_pending; // the search-direction update used partial sums whose finish is still due
    int x_pending;    // multi-RHS CG: this iteration's r update ran, x += alpha p is due (set by the
                      // beta finish, done by the search-direction update, cleared by the next alpha finish)
    double result[4]; // scratch results of standalone reductions
};
enum { kDoneRunning = 0, kDoneStop = 1, kDoneBreakdown = 2, kDoneMaxIter = 3 };

// BiCGStab scalars (complex values as (re, im)); done uses the codes above.
struct BiState {
    double rho[2], alpha[2], omega[2], beta[2];
    double rr, stop_rr;
    int iter, max_iter, done, pad;
};

// Deterministic two-pass reductions.  Pass 1: every block stores the sums of
// its threads' values (in a fixed order) to partials[bid * N + i].  Pass 2
// (a later launch, so the partials are visible without device-wide fences):
// one block of kBlock threads adds the partials in a fixed order.
template <int N, int BS = kBlock>
__device__ __forceinline__ void block_partial(const double (&v)[N], double* partials, int bid) {
    constexpr int kW = BS / 64;
    __shared__ double sh[N][kW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double s = wave_sum(v[i]);
        if (lane == 0) sh[i][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double s = 0;
#pragma unroll
            for (int w = 0; w < kW; ++w) s += sh[i][w];
            partials[(int64_t)bid * N + i] = s;
        }
    }
}

// Pass 2, for a block of BS threads: the totals, in every thread.
template <int N, int BS = kBlock>
__device__ __forceinline__ void sum_partials(const double* partials, int nblocks, double (&tot)[N]) {
    constexpr int kW = BS / 64;
    double acc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = 0;
    // eight independent loads in flight, added in the fixed order b = tid, tid + kBlock, ...
    constexpr int kBatch = 8;
    for (int b0 = threadIdx.x; b0 < nblocks; b0 += kBatch * BS) {
        double v[kBatch][N];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int b = b0 + k * BS;
#pragma unroll
            for (int i = 0; i < N; ++i) v[k][i] = b < nblocks ? partials[(int64_t)b * N + i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k)
#pragma unroll
            for (int i = 0; i < N; ++i) acc[i] += v[k][i];
    }
    __shared__ double sh[N][kW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double s = wave_sum(acc[i]);
        if (lane == 0) sh[i][wave] = s;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double s = 0;
#pragma unroll
        for (int w = 0; w < kW; ++w) s += sh[i][w];
        tot[i] = s;
    }
}

// The solver-scalar update that finishes a CG reduction (one thread):
// kind 0 (alpha): pAp = total, alpha = rr / pAp, breakdown unless pAp > 0;
// kind 1 (beta):  rr_prev = rr, rr = total, beta = rr / rr_prev, iter + 1 and
// the stop tests.
__device__ __forceinline__ void cg_finish_update(CgState* st, double total, int kind) {
    if (kind == 0) {
        st->pAp = total;
        if (!(total > 0.0) || !isfinite(total)) st->done = kDoneBreakdown;
        else st->alpha = st->rr / total;
    } else {
        const double rr_old = st->rr;
        st->rr_prev = rr_old;
        st->rr = total;
        st->beta = total / rr_old;
        const int it = st->iter + 1;
        st->iter = it;
        if (!isfinite(total)) st->done = kDoneBreakdown;
        else if (total <= st->stop_rr || it >= st->cycle_end) st->done = kDoneStop;
        else if (it >= st->max_iter) st->done = kDoneMaxIter;
    }
}

// Whether the solve behind st has stopped, read once per block so that every
// wave of the block takes the same branch (another block of the same launch may
// set the flag meanwhile).  Callable inside a loop: the second barrier keeps the
// next call's write behind every wave's read.
__device__ __forceinline__ bool block_stopped(const CgState* st) {
    __shared__ int flag;
    if (threadIdx.x == 0) flag = st->done;
    __syncthreads();
    const bool stopped = flag != 0;
    __syncthreads();
    return stopped;
}

// A whole block finishes a CG reduction of n partials unless the solve has
// stopped; returns (in every thread) whether the solve is stopped afterwards.
// kind 2 (kFinishBetaPending in internal.h): the beta finish of an iteration whose
// search-direction update already formed beta from the same partials, done only
// when st->beta_pending is set (and then cleared).
template <int BS>
__device__ __forceinline__ bool cg_finish_block(CgState* st, const double* partials, int n, int kind) {
    __shared__ int stopped, skip;
    if (threadIdx.x == 0) {
        stopped = st->done;
        skip = kind == 2 && !st->beta_pending;
        if (kind == 0) st->x_pending = 0;   // the previous iteration's x update has run
    }
    __syncthreads();
    const bool before = stopped != 0, nothing = skip != 0;
    __syncthreads();   // every wave has read the flags before they are written again
    if (before) return true;
    if (nothing) return false;
    double tot[1];
    sum_partials<1, BS>(partials, n, tot);
    if (threadIdx.x == 0) {
        cg_finish_update(st, tot[0], kind == 2 ? 1 : kind);
        if (kind == 2) st->beta_pending = 0;
        if (kind == 1) st->x_pending = 1;
        stopped = st->done;
    }
    __syncthreads();
    const bool after = stopped != 0;
    __syncthreads();   // as above: the batched kernel may call this again in its loop
    return after;
}

}  // namespace tmqcd
