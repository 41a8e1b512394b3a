// Single-RHS hop launches: the kernel template per precision, link format,
// daggering, own term and epilogue, in the launch shape chosen by the tuner.
#include <cstring>

#include "stencil.h"

namespace tmqcd {
using namespace stencil;
namespace {

// BS threads per block and the block order are tuning choices (block_site).
template <int P, int R, bool DAG, bool OWN, int EPI, int PV, int BS>
__global__ __launch_bounds__(BS) void hop_kernel(const HopK a) {
    static_assert(std::is_same<typename Prec<P>::T, typename Prec<PV>::T>::value,
                  "vector and dslash compute types differ");
    if (a.fin_n > 0 && blockIdx.x == 0) {
        if (cg_finish_block<BS>(a.st, a.fin_partials, a.fin_n, a.fin_kind)) return;
    } else if (a.st != nullptr && block_stopped(a.st)) {
        return;   // a solver stage queued after its stop
    }
    int par, h;
    const bool valid = block_site(a, blockIdx.x, threadIdx.x, par, h);
    const double red = valid ? hop_site<P, R, DAG, OWN, EPI, PV>(a, par, h) : 0.0;
    hop_reduce<EPI, BS>(a, red, blockIdx.x);
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
    if (a.nrhs > 1) return launch_hop_mrhs(a, k, s);
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

// the largest grid over block sizes and orders (bounds the reduction partials)
int hop_blocks(const Geom& g, int nparity) {
    HopParams a;
    std::memset(&a, 0, sizeof(a));
    a.g = g;
    a.nparity = 1;
    a.prec = TMQCD_F64;
    int most = 0;
    for (int prec = TMQCD_F64; prec <= TMQCD_F16; ++prec)
        for (int order = 0; order < kNumOrders; ++order) {
            a.prec = prec;
            a.order = order;
            const HopK k = make_hopk(a, kMinBlock);
            most = k.nb_half > most ? k.nb_half : most;
        }
    return nparity * most;
}

int mrhs_tiles_max(const Geom& g, int nparity) {
    HopParams a;
    std::memset(&a, 0, sizeof(a));
    a.g = g;
    a.nparity = nparity;
    a.nrhs = 2;
    int most = 0;
    for (int prec = TMQCD_F64; prec <= TMQCD_F16; ++prec)
        for (int order = 0; order < kNumOrders; ++order) {
            a.prec = prec;
            a.order = order;
            const HopK k = make_hopk(a, 64);
            most = k.nblocks > most ? k.nblocks : most;
        }
    return most;
}

hipError_t launch_hop(const HopParams& a_in, hipStream_t s, int* nblocks) {
    HopParams a = a_in;
    if (a.block == 0) {   // not chosen by the caller: the tuned choice, else the default shape
        TuneChoice t;
        if (tune_lookup(a, &t)) {
            a.block = t.block;
            a.order = t.order;
            a.group = t.group;
        } else {
            // 256 threads; the multi-RHS kernel in t-slab order (its 12 fields per site need the
            // t-neighbours in flight), the others remapped per XCD
            a.block = 256;
            a.order = a.nrhs > 1 ? kOrderSlab : kOrderXcdRemap;
        }
    }
    if (a.block != 128 && a.block != 256) return hipErrorInvalidValue;
    const HopK k = make_hopk(a, a.nrhs > 1 ? 64 : a.block);
    if (nblocks) *nblocks = k.nblocks;   // multi-RHS: tiles per column (its reduction partials per column)
    const int want_vprec = a.prec == TMQCD_F64 ? TMQCD_F64 : TMQCD_F32;
    if (a.epi == kEpiCgUpdate && a.vprec != want_vprec) return hipErrorInvalidValue;
    return with_link_format(a.prec, a.recon, [&](auto p, auto r) {
        return dispatch_variant<decltype(p)::value, decltype(r)::value>(a, k, s);
    });
}

}  // namespace tmqcd
