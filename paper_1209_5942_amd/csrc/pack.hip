// Conversion between the canonical array-of-structures layouts and the packed
// structure-of-arrays layouts (the paper's transparent AoS <-> SoA conversion
// when fields move onto or off the device), with precision conversion and
// 12-real link compression.
#include "device.h"
#include "internal.h"

namespace tmqcd {
namespace {

struct PackK {
    int L[4];
    int64_t vol, vh, stride, gstride, hbytes;
};

__device__ __forceinline__ int parity_of(const PackK& k, int64_t s) {
    const int64_t x = s % k.L[0];
    int64_t r = s / k.L[0];
    const int64_t y = r % k.L[1];
    r /= k.L[1];
    const int64_t z = r % k.L[2];
    const int64_t t = r / k.L[2];
    return (int)((x + y + z + t) & 1);
}

template <int P, int R>
__global__ __launch_bounds__(kBlock) void pack_gauge_kernel(PackK k, const double2* canon, char* packed) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= k.vol) return;
    const int par = parity_of(k, s);
    const int64_t h = s >> 1;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        Su3<double> u;
        const double2* src = canon + (s * 4 + mu) * 9;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            const double2 w = src[e];
            u.m[e / 3][e % 3] = {w.x, w.y};
        }
        LinkIO<P, R>::store(packed, k.gstride, par, mu, h, u);
    }
}

template <int P, int R>
__global__ __launch_bounds__(kBlock) void unpack_gauge_kernel(PackK k, double2* canon, const char* packed) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= k.vol) return;
    const int par = parity_of(k, s);
    const int64_t h = s >> 1;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        Su3<typename Prec<P>::T> u;
        LinkIO<P, R>::load(u, packed, k.gstride, par, mu, h);
        double2* dst = canon + (s * 4 + mu) * 9;
#pragma unroll
        for (int e = 0; e < 9; ++e) dst[e] = make_double2((double)u.m[e / 3][e % 3].re, (double)u.m[e / 3][e % 3].im);
    }
}

// canonical site index i of field `rhs` <-> (half, h) of the packed field
template <int P, bool UNPACK>
__global__ __launch_bounds__(kBlock) void pack_spinor_kernel(PackK k, double2* canon, char* packed, int subset,
                                                             int64_t n, int64_t fbytes) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int rhs = blockIdx.y;
    if (i >= n) return;
    int half;
    int64_t h;
    if (subset == TMQCD_FULL) {
        half = parity_of(k, i);
        h = i >> 1;
    } else {
        half = 0;
        h = i;
    }
    char* hf = packed + rhs * fbytes + half * k.hbytes;
    double2* c = canon + (rhs * n + i) * 12;
    using T = typename Prec<P>::T;
    Spinor<T> v;
    if constexpr (!UNPACK) {
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            const double2 w = c[e];
            v.s[e / 3][e % 3] = {(T)w.x, (T)w.y};
        }
        SpinorIO<P>::store(hf, k.stride, h, v);
    } else {
        SpinorIO<P>::load(v, hf, k.stride, h);
#pragma unroll
        for (int e = 0; e < 12; ++e) c[e] = make_double2((double)v.s[e / 3][e % 3].re, (double)v.s[e / 3][e % 3].im);
    }
}

PackK make_packk(const Geom& g, int prec) {
    PackK k;
    for (int i = 0; i < 4; ++i) k.L[i] = g.L[i];
    k.vol = 2 * g.vh;
    k.vh = g.vh;
    k.stride = g.stride;
    k.gstride = g.gstride;
    k.hbytes = half_field_bytes(g, prec);
    return k;
}

}  // namespace

hipError_t launch_pack_gauge(const Geom& g, const void* canon, void* packed, int prec, int recon, hipStream_t s) {
    const PackK k = make_packk(g, prec);
    const dim3 grid((unsigned)((k.vol + kBlock - 1) / kBlock));
    const double2* c = static_cast<const double2*>(canon);
    char* p = static_cast<char*>(packed);
    return with_link_format(prec, recon, [&](auto pp, auto rr) {
        hipLaunchKernelGGL((pack_gauge_kernel<decltype(pp)::value, decltype(rr)::value>), grid, dim3(kBlock), 0, s, k,
                           c, p);
        return hipGetLastError();
    });
}

hipError_t launch_unpack_gauge(const Geom& g, const void* packed, void* canon, int prec, int recon, hipStream_t s) {
    const PackK k = make_packk(g, prec);
    const dim3 grid((unsigned)((k.vol + kBlock - 1) / kBlock));
    double2* c = static_cast<double2*>(canon);
    const char* p = static_cast<const char*>(packed);
    return with_link_format(prec, recon, [&](auto pp, auto rr) {
        hipLaunchKernelGGL((unpack_gauge_kernel<decltype(pp)::value, decltype(rr)::value>), grid, dim3(kBlock), 0, s,
                           k, c, p);
        return hipGetLastError();
    });
}

hipError_t launch_pack_spinor(const Geom& g, const void* canon, void* packed, int prec, int subset, int nrhs,
                              bool unpack, hipStream_t s) {
    const PackK k = make_packk(g, prec);
    const int64_t n = subset == TMQCD_FULL ? 2 * g.vh : g.vh;
    const int64_t fbytes = field_bytes(g, prec, subset);
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock), (unsigned)nrhs);
    double2* c = const_cast<double2*>(static_cast<const double2*>(canon));
    char* p = static_cast<char*>(packed);
#define TMQCD_PACK(PR)                                                                                         \
    if (prec == PR) {                                                                                          \
        if (unpack) hipLaunchKernelGGL((pack_spinor_kernel<PR, true>), grid, dim3(kBlock), 0, s, k, c, p, subset, n, fbytes); \
        else hipLaunchKernelGGL((pack_spinor_kernel<PR, false>), grid, dim3(kBlock), 0, s, k, c, p, subset, n, fbytes);       \
        return hipGetLastError();                                                                              \
    }
    TMQCD_PACK(TMQCD_F64)
    TMQCD_PACK(TMQCD_F32)
    TMQCD_PACK(TMQCD_F16)
#undef TMQCD_PACK
    return hipErrorInvalidValue;
}

}  // namespace tmqcd
