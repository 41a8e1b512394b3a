// Operator composition and solver drivers (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tmqcd {

extern thread_local int g_last_hip_error;

struct OpCtx {
    Geom g;
    int prec, recon;
    const void* gauge;
    hipStream_t s;
    double kappa, w;   // w = 2 kappa mu
    Cplx bc[4];
};

OpCtx make_ctx(const tmqcd_problem& prob, int prec, int recon, const void* gauge, hipStream_t s);

// several right-hand sides: count and byte strides between consecutive fields
struct Rhs {
    int n;
    int64_t in, own, out;
};
static const Rhs kOne = {1, 0, 0, 0};

// launch parameters of the two halves of the Schur complement (see ops.cpp)
HopParams hp_schur_first(const OpCtx& c, const void* in_e, void* t_o, bool dag, const Rhs& r);
HopParams hp_schur_second(const OpCtx& c, const void* t_o, const void* own_e, void* out_e, bool dag, int epi,
                          CgState* st, double* partials, void* x, void* r, const void* p, const Rhs& rh);

// full field: out = A(+-mu) in - kappa H(^+) in, with the epilogue epi (see ops.cpp)
HopParams hp_full(const OpCtx& c, const void* in, void* out, bool dag, int epi, CgState* st, double* partials,
                  void* x, void* r, const void* p, const Rhs& rh);

// out = op(in) for nrhs consecutive fields; tmp must hold nrhs * dslash_tmp_bytes(g, op, prec) bytes
hipError_t apply_operator(const OpCtx& c, int op, const void* in, void* out, char* tmp, int nrhs);
int64_t dslash_tmp_bytes(const Geom& g, int op, int prec);

// The even-odd fermion force (see ops.cpp): scale * G written into or added to out;
// X_e: packed FP64 even field; tmp: force_eo_tmp_bytes(g) bytes.  c.prec must be FP64.
hipError_t force_eo(const OpCtx& c, const void* X_e, double* out, double scale, int accumulate, char* tmp);
int64_t force_eo_tmp_bytes(const Geom& g);

struct CgWorkspace {
    CgState* st;
    double* partials;                         // the alpha reductions (and standalone ones)
    double* partials_b;                       // the beta reductions of the update hop
    void *r, *p, *ax, *t1, *t2, *t3;          // FP64
    void *rs, *xs, *ps, *t1s, *t2s, *t3s;     // inner precision (mixed)
    int64_t total;
};
// Layout of the CG workspace; with base == nullptr only `total` is meaningful.
CgWorkspace carve_cg(const Geom& g, int op, int inner_prec, char* base);
int64_t state_bytes();
int64_t partial_bytes(const Geom& g);

// CG on Mhat^+ Mhat for n lattices at once (FP64): every stage of an iteration
// is one launch over all lattices; with use_graph one iteration is captured in
// a hipGraph and replayed.  stats[n]; b, x: packed FP64 even fields.
int run_cg_batch(int n, const tmqcd_problem* probs, const void* const* gauge, const void* const* b, void* const* x,
                 const tmqcd_cg_opts& o, tmqcd_cg_stats* stats, bool use_graph, void* ws, hipStream_t s);
int64_t cg_batch_workspace(int n, const tmqcd_problem* probs);

// autotuning (tune.cpp)
int64_t tune_workspace_bytes(const Geom& g, int prec);
int run_tune(const tmqcd_problem& prob, const void* gauge, int prec, int recon, void* ws, hipStream_t s,
             tmqcd_tune_result results[3]);
int tune_save(const char* path);
int tune_load(const char* path);
void tune_clear();
void tune_set(const tmqcd_problem& prob, int prec, int recon, int cls, int nrhs, int block, int order, int group);
bool valid_choice(int cls, int nrhs, int block, int order, int group);
int64_t tune_mrhs_workspace_bytes(const Geom& g, int prec, int nrhs);
int run_tune_mrhs(const tmqcd_problem& prob, const void* gauge, int prec, int recon, int nrhs, void* ws,
                  hipStream_t s, tmqcd_tune_result* res);

// BiCGStab on M (full field) or Mhat (even field) in FP64 (bicgstab.hip); o.op selects
// the operator, o.recon the links; workspace bicgstab_workspace(g, op) bytes.
int run_bicgstab(const tmqcd_problem& prob, const void* gauge, const void* b, void* x, const tmqcd_cg_opts& o,
                 tmqcd_cg_stats& stats, void* ws, hipStream_t s);
int64_t bicgstab_workspace(const Geom& g, int op);

int run_cg(const tmqcd_problem& prob, const void* const gauge[3], const void* b, void* x, const tmqcd_cg_opts& o,
           tmqcd_cg_stats& stats, void* ws, hipStream_t s);

// CG on o.nrhs > 1 right-hand sides at once (FP64; cg_mrhs.cpp): b, x hold o.nrhs packed fields one after
// the other, stats[o.nrhs]; workspace carve_cg_mrhs(g, op, n, nullptr).total bytes
struct MrhsWorkspace {
    CgState* st;                 // CgState[n]
    double* partials;            // [n][tiles_max]: the multi-RHS launches' per-column sums
    double* setup_partials;      // [n][col_partials]: per-column set-up and residual reductions
    char *r, *p, *ax, *t1, *t2;  // n columns each, fstride bytes apart (t1, t2: the operator's temporaries)
    int64_t fstride, tiles_max, col_partials, total;
};
MrhsWorkspace carve_cg_mrhs(const Geom& g, int op, int n, char* base);
int run_cg_mrhs(const tmqcd_problem& prob, const void* gauge, const void* b, void* x, const tmqcd_cg_opts& o,
                tmqcd_cg_stats* stats, void* ws, hipStream_t s);

}  // namespace tmqcd
