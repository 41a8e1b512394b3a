// Packed device layouts and lattice geometry (host and device).
//
// Structure-of-arrays over the sites of one parity with a 16-byte base type,
// as the paper's storage-format study found best for bandwidth: a site's
// components are spread over `units` arrays, each `stride` elements long, so
// that consecutive lanes of a wavefront read consecutive 16-byte words.  Links
// are split by the parity of their origin site so that an even-odd hop never
// reads links it does not use.
//
//   spinor half field, per precision (stride = site count rounded up to 64):
//     F64: 12 x double2          [12][stride]   one complex per unit
//     F32:  6 x float4           [ 6][stride]   two complexes per unit
//     F16:  3 x 8 halves (16 B)  [ 3][stride]   four complexes per unit,
//           followed by float    [stride]       per-site scale
//   full field = even half, then odd half; nrhs fields follow each other.
//
//   gauge field: [parity of origin][mu][unit][gstride], unit type per (prec, recon):
//     F64 R18: 9 x double2   R12: 6 x double2  (rows 0 and 1)
//     F32 R18: 9 x float2    R12: 3 x float4
//     F16 R18: 9 x half2     R12: 3 x (4 halves, 8 B)
#pragma once

#include <cstddef>
#include <cstdint>

#include "tmqcd.h"

namespace tmqcd {

constexpr int64_t kAlignSites = 64;    // one wavefront
constexpr int64_t kAlignBytes = 256;

__host__ __device__ inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Geom {
    int L[4];          // Lx, Ly, Lz, Lt
    int lxh;           // Lx / 2
    int64_t vh;        // sites per parity
    int64_t stride;    // spinor SoA stride (elements)
    int64_t gstride;   // gauge SoA stride (elements)
};

inline Geom make_geom(const tmqcd_problem& p) {
    Geom g;
    for (int i = 0; i < 4; ++i) g.L[i] = p.dims[i];
    g.lxh = p.dims[0] / 2;
    g.vh = (int64_t)p.dims[0] * p.dims[1] * p.dims[2] * p.dims[3] / 2;
    g.stride = round_up(g.vh, kAlignSites);
    g.gstride = round_up(g.vh, kAlignSites);
    return g;
}

// bytes of one packed half field of precision `prec`
inline int64_t half_field_bytes(const Geom& g, int prec) {
    int64_t b = 0;
    switch (prec) {
        case TMQCD_F64: b = 12 * 16 * g.stride; break;
        case TMQCD_F32: b = 6 * 16 * g.stride; break;
        case TMQCD_F16: b = 3 * 16 * g.stride + 4 * g.stride; break;
        default: return 0;
    }
    return round_up(b, kAlignBytes);
}

inline int64_t field_bytes(const Geom& g, int prec, int subset) {
    return (subset == TMQCD_FULL ? 2 : 1) * half_field_bytes(g, prec);
}

// gauge: number of storage units per link and bytes per unit
inline int gauge_units(int prec, int recon) {
    switch (recon) {
        case TMQCD_RECON18: return 9;
        case TMQCD_RECON12: return prec == TMQCD_F64 ? 6 : 3;
        case TMQCD_RECON10: return 5;
        case TMQCD_RECON8: return prec == TMQCD_F64 ? 4 : (prec == TMQCD_F32 ? 2 : 1);
    }
    return 0;
}
inline int gauge_unit_bytes(int prec, int recon) {
    switch (prec) {
        case TMQCD_F64: return 16;
        case TMQCD_F32: return (recon == TMQCD_RECON18 || recon == TMQCD_RECON10) ? 8 : 16;
        case TMQCD_F16: return (recon == TMQCD_RECON18 || recon == TMQCD_RECON10) ? 4 : (recon == TMQCD_RECON12 ? 8 : 16);
    }
    return 0;
}
inline int64_t gauge_bytes(const Geom& g, int prec, int recon) {
    return round_up(2 * 4 * (int64_t)gauge_units(prec, recon) * gauge_unit_bytes(prec, recon) * g.gstride,
                    kAlignBytes);
}

}  // namespace tmqcd
