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

// out = op(in); tmp must hold dslash_tmp_bytes(g, op, prec) bytes
hipError_t apply_operator(const OpCtx& c, int op, const void* in, void* out, char* tmp);
int64_t dslash_tmp_bytes(const Geom& g, int op, int prec);

struct CgWorkspace {
    CgState* st;
    double* partials;
    void *r, *p, *ax, *t1, *t2, *t3;          // FP64
    void *rs, *xs, *ps, *t1s, *t2s, *t3s;     // inner precision (mixed)
    int64_t total;
};
// Layout of the CG workspace; with base == nullptr only `total` is meaningful.
CgWorkspace carve_cg(const Geom& g, int op, int inner_prec, char* base);
int64_t state_bytes();
int64_t partial_bytes(const Geom& g);

int run_cg(const tmqcd_problem& prob, const void* const gauge[3], const void* b, void* x, const tmqcd_cg_opts& o,
           tmqcd_cg_stats& stats, void* ws, hipStream_t s);

}  // namespace tmqcd
