// Several lattices in one hop launch (the batched multi-lattice CG).
#include "stencil.h"

namespace tmqcd {
using namespace stencil;
namespace {

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
        if (a.fin_n > 0 && tile == b.tile_start[i]) {   // the lattice's first tile finishes its reduction
            if (cg_finish_block<kBlock>(a.st, a.fin_partials, a.fin_n, a.fin_kind)) continue;
        } else if (a.st != nullptr && block_stopped(a.st)) {
            continue;   // block-uniform: every wave skips the tile together
        }
        const int lt = tile - b.tile_start[i];
        int par, h;
        const bool valid = block_site(a, lt, threadIdx.x, par, h);
        const double red = valid ? hop_site<P, R, DAG, OWN, EPI, PV>(a, par, h) : 0.0;
        hop_reduce<EPI>(a, red, lt);
        __syncthreads();   // the reduction's shared memory is reused by the next tile
    }
}

template <int R, bool DAG, bool OWN, int EPI>
hipError_t launch_batch_inst(const HopBatch& b, int grid, hipStream_t s) {
    hipLaunchKernelGGL((hop_batch_kernel<TMQCD_F64, R, DAG, OWN, EPI, TMQCD_F64>), dim3(grid), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}
template <bool DAG, bool OWN, int EPI>
hipError_t launch_batch_recon(int recon, const HopBatch& b, int grid, hipStream_t s) {
    switch (recon) {
        case TMQCD_RECON18: return launch_batch_inst<TMQCD_RECON18, DAG, OWN, EPI>(b, grid, s);
        case TMQCD_RECON12: return launch_batch_inst<TMQCD_RECON12, DAG, OWN, EPI>(b, grid, s);
        case TMQCD_RECON10: return launch_batch_inst<TMQCD_RECON10, DAG, OWN, EPI>(b, grid, s);
        case TMQCD_RECON8: return launch_batch_inst<TMQCD_RECON8, DAG, OWN, EPI>(b, grid, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_hop_batch(const HopParams* ps, int n, int max_grid, hipStream_t s, int* nblocks) {
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
        a256.order = kOrderLinear;
        b.lat[i] = make_hopk(a256, kBlock);
        b.tile_start[i + 1] = b.tile_start[i] + b.lat[i].nblocks;
        if (nblocks) nblocks[i] = b.lat[i].nblocks;
    }
    const int total = b.tile_start[n];
    const int grid = total < max_grid ? total : max_grid;
    const HopParams& a = ps[0];
    const bool own = a.own != nullptr;
#define TMQCD_BATCH(D, O, E) return launch_batch_recon<D, O, E>(a.recon, b, grid, s)
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
