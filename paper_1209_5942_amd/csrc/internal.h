// Host-side interfaces between the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "layout.h"

namespace tmqcd {

struct CgState;   // device.h

struct Cplx {
    double re, im;
};

// Epilogue kinds of the hop kernel.
enum HopEpilogue {
    kEpiStore = 0,      // out = own-term + hop-term
    kEpiStoreNorm = 1,  // ... and the partial sums of |out|^2 (then cg_finish: pAp, alpha)
    kEpiCgUpdate = 2,   // out not stored: r -= alpha out (and x += alpha p where x is given: the batched CG);
                        // partial sums of |r|^2 (cg_finish: rr, beta)
};

// out_p = [c_own * own_p] + c_hop * (H in)_p, where c = diag(cu, cu, cd, cd) in
// spin (upper / lower chiral halves), H is the hop (or H^dagger when dag), and
// p runs over one output parity (nparity = 1; in is the half field of the
// other parity) or both (nparity = 2; in, own and out are full fields).
struct HopParams {
    Geom g;
    int prec, recon;
    const void* gauge;
    const void* in;
    const void* own;
    void* out;
    int out_parity;
    int nparity;
    bool dag;
    Cplx bc[4];
    Cplx cu_own, cd_own, cu_hop, cd_hop;
    int epi;
    // reductions and CG update (epi != kEpiStore); with st set, the launch returns at once once st->done
    CgState* st;
    double* partials;
    void* x;          // vector precision
    void* r;          // vector precision
    const void* p;    // dslash precision
    int vprec;        // precision of x and r
    // several right-hand sides: fields nrhs apart by these byte strides; inside the multi-RHS CG
    // (FP64; st points at nrhs states, partials holds nrhs x tiles sums) the vector fields x, r, p
    // are v_fstride apart
    int nrhs;
    int64_t in_fstride, own_fstride, out_fstride, v_fstride;
    // launch shape: block 128 or 256 threads and the block order (kOrder*); block = 0 takes the tuned choice;
    // group: right-hand sides per block of the multi-RHS kernel (0: all)
    int block;
    int order;
    int group;
    // fin_n > 0: block 0 first finishes the CG reduction of the previous launch (fin_n partials,
    // kind fin_kind of launch_cg_finish) on st
    const double* fin_partials;
    int fin_n, fin_kind;
};

// Block orders of the hop launches (which sites a block covers, see block_site in stencil.h).
// kOrderSlab, kOrderSlabT2, kOrderSlabT4: each XCD owns one of (8, 4, 2) z-ranges of the t-slices of one of
// (1, 2, 4) t-ranges and walks through its t-range (see block_site).
enum BlockOrder {
    kOrderLinear = 0, kOrderXcdRemap = 1, kOrderSlab = 2, kOrderColumn = 3, kOrderSlabT2 = 4, kOrderSlabT4 = 5,
    kNumOrders = 6
};
__host__ __device__ inline bool slab_order(int order) { return order == kOrderSlab || order == kOrderSlabT2 || order == kOrderSlabT4; }

constexpr int kMaxRhs = 16;   // right-hand sides of one multi-RHS launch

// ---- autotuning (tune.cpp) ------------------------------------------------------
// kernel classes: 0 hop (store), 1 hop + |out|^2, 2 hop + CG update, 3 multi-RHS hop
constexpr int kClassMultiRhs = 3;
struct TuneChoice {
    int block;
    int order;
    int group;   // multi-RHS class: right-hand sides per block (0: all)
    double us;
};
// the tuned launch shape for this hop (class from epi, or the multi-RHS class with its nrhs)
bool tune_lookup(const HopParams& a, TuneChoice* out);

// *nblocks (if given): the number of blocks, i.e. of reduction partials this launch writes
hipError_t launch_hop(const HopParams& a, hipStream_t s, int* nblocks = nullptr);
// one launch over the same stage for n <= 8 lattices (FP64), grid-stride over their tiles;
// nblocks[i] (if given): the number of reduction partials lattice i receives
hipError_t launch_hop_batch(const HopParams* ps, int n, int max_grid, hipStream_t s, int* nblocks = nullptr);
int hop_blocks(const Geom& g, int nparity);   // grid size (and partial count) of a hop launch
int mrhs_tiles_max(const Geom& g, int nparity);   // tiles of a multi-RHS launch (its partials per column)

// ---- BLAS-1 over packed fields of nhalf half fields -------------------------
// Calls f(integral_constant<P>, integral_constant<R>) for the run-time storage precision and
// link encoding (every combination is compiled); hipErrorInvalidValue for an unknown pair.
template <typename F>
hipError_t with_link_format(int prec, int recon, F&& f) {
    using std::integral_constant;
#define TMQCD_LF(P, R) \
    if (prec == P && recon == R) return f(integral_constant<int, P>{}, integral_constant<int, R>{});
#define TMQCD_LF_R(P) TMQCD_LF(P, TMQCD_RECON18) TMQCD_LF(P, TMQCD_RECON12) TMQCD_LF(P, TMQCD_RECON10) TMQCD_LF(P, TMQCD_RECON8)
    TMQCD_LF_R(TMQCD_F64)
    TMQCD_LF_R(TMQCD_F32)
    TMQCD_LF_R(TMQCD_F16)
#undef TMQCD_LF_R
#undef TMQCD_LF
    return hipErrorInvalidValue;
}

struct VecSpec {
    const Geom* g;
    int nhalf;       // 1 = half field, 2 = full field
};
// dst = src (precision conversion, rounding to nearest)
hipError_t launch_convert(const VecSpec& v, void* dst, int pdst, const void* src, int psrc, hipStream_t s);
// st->result[slot] = |src|^2 (deterministic FP64 reduction)
hipError_t launch_norm2(const VecSpec& v, const void* src, int prec, CgState* st, int slot, double* partials,
                        hipStream_t s);
// r = b - ax (all FP64), st->result[slot] = |r|^2
hipError_t launch_residual(const VecSpec& v, void* r, const void* b, const void* ax, CgState* st, int slot,
                           double* partials, hipStream_t s);
// p = r + beta p with beta = st->beta; nothing when st->done and skip_if_done
hipError_t launch_xpay(const VecSpec& v, void* p, int pp, const void* r, int pr, CgState* st, bool skip_if_done,
                       hipStream_t s);
// p = r + beta p with beta = (sum of the n partials) / st->rr formed by every block in a fixed order
// (the partials of the update hop's |r|^2); sets st->beta_pending; nothing once st->done
hipError_t launch_xpay_fused(const VecSpec& v, void* p, int pp, const void* r, int pr, void* x, CgState* st,
                             const double* partials, int n, hipStream_t s);
// For n <= 8 lattices (FP64 even fields), as launch_xpay_fused for each: beta from the np[i]
// partials of the update hop, x += alpha p, p = r + beta p unless this iteration stops the
// lattice; sets st[i]->beta_pending; nothing for a lattice whose solve has stopped
hipError_t launch_xpay_batch(const VecSpec* vs, void* const* p, const void* const* r, void* const* x,
                             CgState* const* st, const double* const* partials, const int* np, int n, int max_grid,
                             hipStream_t s);
// x64 += xs (low precision), then xs = 0
hipError_t launch_accumulate(const VecSpec& v, void* x64, void* xs, int ps, hipStream_t s);
hipError_t launch_zero(const VecSpec& v, void* dst, int prec, hipStream_t s);
// deterministic test values; count of differing 8-byte words (added to *mismatches)
hipError_t launch_fill(const VecSpec& v, void* dst, int prec, unsigned seed, hipStream_t s);
hipError_t launch_compare(const void* a, const void* b, int64_t bytes, unsigned long long* mismatches, hipStream_t s);

// ---- solver state --------------------------------------------------------------
struct StateInit {
    double rr, rr_prev, stop_rr, alpha, beta;
    int iter, max_iter, cycle_end, done;
    bool set_rr, set_rr_prev, set_stop, set_alpha, set_beta, set_iter, set_max_iter, set_cycle_end, set_done;
};
hipError_t launch_set_state(CgState* st, const StateInit& v, hipStream_t s);
// Second pass of a CG reduction over n partials (one block per lattice):
//   kFinishAlpha: pAp = sum, alpha = rr / pAp (done = breakdown unless pAp > 0)
//   kFinishBeta:  rr_prev = rr, rr = sum, beta = rr / rr_prev, iter + 1, stop tests
//   kFinishBetaPending: kFinishBeta if st->beta_pending (then cleared), else nothing: the CG
//                 iteration forms beta in its search-direction update (launch_xpay_fused) and
//                 leaves this finish to the next launch that carries it
// Nothing happens for a lattice whose st->done is set.
enum FinishKind { kFinishAlpha = 0, kFinishBeta = 1, kFinishBetaPending = 2 };
hipError_t launch_cg_finish(CgState* st, const double* partials, int n, int kind, hipStream_t s);
hipError_t launch_cg_finish_batch(CgState* const* st, const double* const* partials, const int* n, int count,
                                  int kind, hipStream_t s);
// The multi-RHS CG: column c's reduction (tiles partials at partials + c * tiles) finished on st[c]
// for c < ncol; x_c += alpha_c p_c for the columns whose r update ran in this iteration
// (st[c].x_pending), then p_c = r_c + beta_c p_c for the running columns (FP64 fields fstride
// bytes apart)
hipError_t launch_cg_finish_cols(CgState* st, const double* partials, int tiles, int ncol, int kind, hipStream_t s);
hipError_t launch_xpay_cols(const VecSpec& v, void* p, const void* r, void* x, int64_t fstride, int ncol,
                            const CgState* st, hipStream_t s);
// st->rr = st->result[slot]; optionally stop_rr = factor * rr
hipError_t launch_rr_from_result(CgState* st, int slot, double stop_factor, hipStream_t s);

// ---- packing ----------------------------------------------------------------------
hipError_t launch_pack_gauge(const Geom& g, const void* canon, void* packed, int prec, int recon, hipStream_t s);
hipError_t launch_unpack_gauge(const Geom& g, const void* packed, void* canon, int prec, int recon, hipStream_t s);
hipError_t launch_pack_spinor(const Geom& g, const void* canon, void* packed, int prec, int subset, int nrhs,
                              bool unpack, hipStream_t s);

// ---- fermion force ---------------------------------------------------------------
// out = scale * G (accumulate = 0) or out += scale * G (accumulate = 1); X[p], Y[p]: the
// parity-p halves of the two FP64 fields (of one full field, or from separate buffers)
hipError_t launch_force(const Geom& g, const void* gauge, int recon, const void* const X[2], const void* const Y[2],
                        double* out, const Cplx bc[4], double kappa, double scale, int accumulate, hipStream_t s);

// ---- bandwidth probe (probe.hip): read (dst == nullptr; xor of the words into *xor_out) or copy
hipError_t launch_hbm_probe(const void* src, void* dst, int64_t bytes, int grid, unsigned* xor_out, hipStream_t s);

// ---- HMC kernels and auxiliary reductions (partials: aux_partials_doubles(g) doubles) ----
int64_t aux_partials_doubles(const Geom& g);
hipError_t launch_gauge_force(const Geom& g, const void* gauge, double beta, double* out, double scale, int accumulate,
                              hipStream_t s);
hipError_t launch_update_links(const Geom& g, void* gauge, const double* mom, double dt, hipStream_t s);
hipError_t launch_plaquette(const Geom& g, const void* gauge, double* result, double* partials, hipStream_t s);
// tree-level Symanzik gauge force (plaquettes with c0 = 1 - 8 c1, rectangles with c1) and the rectangle sum
// (c1 != 0: ws holds staple_field_bytes(g) bytes for the single plaquette staples)
hipError_t launch_gauge_force_sym(const Geom& g, const void* gauge, double beta, double c1, double* out, double scale,
                                  int accumulate, void* ws, hipStream_t s);
int64_t staple_field_bytes(const Geom& g);
hipError_t launch_rectangle(const Geom& g, const void* gauge, double* result, double* partials, hipStream_t s);
// one heatbath (heatbath = true) or overrelaxation sweep of the Wilson plaquette action, in place on the
// packed RECON18 links of precision prec (FP64 or FP32; heatbath.hip)
hipError_t launch_su3_sweep(const Geom& g, void* gauge, int prec, double beta, uint64_t seed, uint32_t sweep,
                            bool heatbath, hipStream_t s);
hipError_t launch_mom_norm2(const Geom& g, const double* mom, double* result, double* partials, hipStream_t s);
hipError_t launch_spinor_dot(const Geom& g, const void* x, const void* y, int nhalf, double* result, double* partials,
                             hipStream_t s);
// result[0..3] = (dH, kinetic, gauge, fermion parts) between (u0, p0, x0) and (u1, p1, x1), summed site by site
// (pseudofermion phi and the solutions x0, x1 on the first fermion_parities halves: 1 even, 2 full)
hipError_t launch_delta_h(const Geom& g, const void* u0, const void* u1, const double* p0, const double* p1,
                          const void* phi, const void* x0, const void* x1, int fermion_parities, double beta, double c1,
                          double* result, double* partials, hipStream_t s);

}  // namespace tmqcd
