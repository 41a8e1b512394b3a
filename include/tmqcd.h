/*
 * tmqcd.h - C interface of the MI355X (gfx950) twisted-mass Wilson library.
 *
 * Operation (Bach, Lindenstruth, Philipsen, Pinke, "Lattice QCD based on
 * OpenCL", arXiv:1209.5942, section 2.1, the definition of D_tm):
 *
 *   M = D_tm^+ = A - kappa*H,   A = 1 + i*2*kappa*mu*gamma5,
 *   (H psi)(x) = sum_mu [ b+_mu(x) (1 - gamma_mu) U_mu(x)       psi(x + mu)
 *                       + b-_mu(x) (1 + gamma_mu) U_mu(x - mu)^+ psi(x - mu) ]
 *
 * The paper prints the hopping prefactor as kappa/2; this library uses kappa
 * (with kappa = 1/(2(am + 4)) the free massless operator then has its zero mode
 * at kappa = 1/8).  b+_mu(x) = bc_mu if x_mu = L_mu - 1 and 1 otherwise;
 * b-_mu(x) = conj(bc_mu) if x_mu = 0 and 1 otherwise: the boundary phase sits
 * only on hops that cross the lattice boundary.  The paper's Dslash is -kappa*H.
 *
 * Conventions
 *   - Site index s = x + Lx*(y + Ly*(z + Lz*t)), x fastest; direction
 *     mu = 0,1,2,3 <-> x,y,z,t.  Parity (x+y+z+t) mod 2, even = 0.  A field on
 *     one parity ("half field") is indexed by h = s >> 1.  All four extents must
 *     be even and >= 2.
 *   - Gamma matrices (the paper fixes only their anticommutator): chiral basis
 *     gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for k = x,y,z,
 *     gamma_t = [[0, -1], [-1, 0]], gamma5 = gamma_x gamma_y gamma_z gamma_t
 *     = diag(-1, -1, +1, +1).  Spin index 0..3 in this basis.
 *   - Canonical (user-visible) layouts, complex128 = two doubles (re, im):
 *       gauge   U[V][4][3][3]   U[s][mu][a][b] = (U_mu(s))_ab, the link s -> s+mu
 *       spinor  psi[V][4][3]    full field, or psi[Vh][4][3] for one parity
 *       multi-RHS fields are [nrhs][...] with the single-field layout inside
 *       force   dSdw[V][4][8]   float64, coefficient of T^a = lambda^a / 2
 *   - Packed (device) layouts are opaque; their sizes come from the *_bytes
 *     queries.  Internally fields are structure-of-arrays over sites with a
 *     16-byte base type, links split by the parity of their origin site (the
 *     paper's storage-format section).  A packed full spinor holds the even
 *     half followed by the odd half.
 *
 * Ownership and streams
 *   - Every pointer argument that names a field is a DEVICE pointer owned by
 *     the caller; the library allocates no device memory for fields or
 *     scratch.  Scratch memory comes from the caller's workspace `ws` of
 *     `ws_bytes` bytes, sized by tmqcd_workspace_bytes (tmqcd_cg_batch with
 *     graphs creates a HIP graph, and on the null stream a stream, and destroys
 *     them before it returns), except for tmqcd_dslash_noalloc, whose scratch is
 *     a static device array of the library.  Problem, option and stats structs
 *     are host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     tmqcd_pack_*, tmqcd_unpack_*, tmqcd_dslash, the forces, the link update,
 *     the reductions, tmqcd_heatbath and tmqcd_overrelax are stream-ordered
 *     and return without waiting.  tmqcd_cg, tmqcd_cg_batch and tmqcd_bicgstab
 *     synchronise the stream (they read residuals back) and return when the
 *     solve has ended.
 *
 * Entry points: sizes and workspaces (*_bytes); packing; tmqcd_dslash (the
 * operators, 1..16 right-hand sides) and tmqcd_dslash_noalloc; solvers tmqcd_cg (CG on M^+M or
 * Mhat^+Mhat, FP64 or mixed precision), tmqcd_cg_batch (several lattices),
 * tmqcd_bicgstab (M or Mhat); HMC pieces tmqcd_force, tmqcd_force_eo,
 * tmqcd_gauge_force, tmqcd_gauge_force_tlsym, tmqcd_update_links,
 * tmqcd_plaquette, tmqcd_rectangle, tmqcd_momentum_norm2, tmqcd_dot, tmqcd_delta_h; pure-gauge
 * updates tmqcd_heatbath and tmqcd_overrelax; the autotuner (tmqcd_tune*);
 * tmqcd_hbm_probe; errors (tmqcd_error_string, tmqcd_last_hip_error).
 *   - No exceptions cross the interface; functions return TMQCD_OK (0) or a
 *     negative error code.  Arguments are validated on the host before any HIP
 *     call, so every argument error is reported without touching the device.
 *     The library keeps no state between calls other than the last HIP error
 *     code of the calling thread and the process-wide table of tuned launch
 *     shapes (see autotuning; guarded by a mutex, so calls from several host
 *     threads are safe).
 */
#ifndef TMQCD_H
#define TMQCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define TMQCD_OK           0
#define TMQCD_EINVAL      -1  /* bad extent, NULL pointer, unknown op/prec/recon, nrhs out of range */
#define TMQCD_EALIAS      -2  /* output overlaps an input it may not overlap */
#define TMQCD_EALIGN      -3  /* a device pointer is not 256-byte aligned */
#define TMQCD_ENOCONV     -4  /* max_iter reached; x holds the last iterate, stats are filled */
#define TMQCD_EBREAKDOWN  -5  /* NaN/Inf residual or p^+ A p <= 0 in CG */
#define TMQCD_EHIP        -6  /* a HIP call failed; see tmqcd_last_hip_error() */
#define TMQCD_EWORKSPACE  -7  /* ws is NULL or smaller than tmqcd_workspace_bytes() */
#define TMQCD_ESCRATCH    -8  /* tmqcd_dslash_noalloc: temporaries exceed the library's static scratch */

/* ---- problem description --------------------------------------------------- */
typedef struct {
    int32_t dims[4];   /* Lx, Ly, Lz, Lt: each even and >= 2 */
    double kappa;      /* hopping parameter */
    double mu;         /* twisted mass a*mu (dimensionless) */
    double bc[4][2];   /* boundary phase (re, im) of direction mu; (1,0) periodic, (-1,0) antiperiodic */
} tmqcd_problem;

/* storage precisions; arithmetic is FP64 for TMQCD_F64 and FP32 otherwise */
#define TMQCD_F64 0
#define TMQCD_F32 1
#define TMQCD_F16 2   /* IEEE half: links unscaled (|U_ab| <= 1), spinors with one FP32 scale per site */

/* link storage (the paper's §4.1, Table 3): all 18 reals; the first two rows
 * (12 reals) with the third rebuilt as conj(row1 x row2), exact for det U = 1
 * (REC12); the first row and first column (10 reals), the other four entries
 * rebuilt from unitarity and det U = 1 (REC10); as REC10 with |a1| and |c1|
 * rebuilt from the unit norms of the first row and column and only their
 * phases stored (8 reals, REC8).  REC10 and REC8 divide by |a2|^2 + |a3|^2 and
 * lose accuracy as the first row approaches a pure phase times (1, 0, 0). */
#define TMQCD_RECON18 0
#define TMQCD_RECON12 1
#define TMQCD_RECON10 2
#define TMQCD_RECON8  3

/* spinor subsets */
#define TMQCD_FULL 0
#define TMQCD_EVEN 1
#define TMQCD_ODD  2

/* operators for tmqcd_dslash (the paper's section 2.1; even-odd preconditioning
 * as the Schur complement on even sites) */
#define TMQCD_DSLASH_EO     0  /* even <- odd:  out_e = -kappa H_eo in_o  */
#define TMQCD_DSLASH_OE     1  /* odd <- even:  out_o = -kappa H_oe in_e  */
#define TMQCD_M             2  /* full:  M = A - kappa H                      */
#define TMQCD_MDAG          3  /* full:  M^+ = A^+ - kappa H^+                */
#define TMQCD_MDAGM         4  /* full:  M^+ M                                */
#define TMQCD_MHAT          5  /* even:  Mhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe */
#define TMQCD_MHATDAG       6  /* even:  Mhat^+                               */
#define TMQCD_MHATDAGMHAT   7  /* even:  Mhat^+ Mhat                          */

/* ---- size queries (host only, never fail: 0 means invalid arguments) -------- */
/* Bytes of a packed gauge field and of nrhs packed spinor fields.  The FP64
 * sizes per site are the paper's Table 3 (its memory-requirements section, 4.1):
 * 576 / 384 / 320 / 256 B of links for REC18 / 12 / 10 / 8 and 192 B per spinor
 * site, plus padding of each array to a wavefront of sites and 256 bytes. */
size_t tmqcd_gauge_bytes(const tmqcd_problem* prob, int prec, int recon);
size_t tmqcd_spinor_bytes(const tmqcd_problem* prob, int prec, int subset, int nrhs);
/* Workspace for tmqcd_dslash (op), tmqcd_cg (op = TMQCD_MDAGM or
 * TMQCD_MHATDAGMHAT; nrhs > 1 for the multi-RHS solve) and the reductions of the
 * HMC helpers (op = -1).  prec_mask: bit (1 << prec) for every storage precision
 * the call will use (for CG: F64 and the inner one).  The temporaries are those
 * of the operator compositions of the paper's section 2.1 (one odd half field per
 * right-hand side between the two hops of Mhat, a full field between M and M^+)
 * and, for CG, the solver's vectors r, p, A p and its reduction partials. */
size_t tmqcd_workspace_bytes(const tmqcd_problem* prob, int op, int prec_mask, int nrhs);

/* ---- layout conversion (the paper's transparent AoS <-> SoA conversion) ----- */
/* Pack a canonical complex128 gauge field U_canon[V][4][3][3] (device) into the
 * packed layout of (prec, recon).  Rounds to nearest even on down-conversion. */
int tmqcd_pack_gauge(const tmqcd_problem* prob, const void* U_canon, void* U_packed,
                     int prec, int recon, void* stream);
/* Inverse of tmqcd_pack_gauge: packed -> canonical complex128 U_canon[V][4][3][3]
 * (12-real links come back with their third row rebuilt). */
int tmqcd_unpack_gauge(const tmqcd_problem* prob, const void* U_packed, void* U_canon,
                       int prec, int recon, void* stream);
/* Pack canonical complex128 spinors [nrhs][n][4][3] (n = V for TMQCD_FULL, V/2
 * otherwise) into the packed layout of prec.  in_canon and out_packed must not
 * overlap. */
int tmqcd_pack_spinor(const tmqcd_problem* prob, const void* in_canon, void* out_packed,
                      int prec, int subset, int nrhs, void* stream);
/* Inverse of tmqcd_pack_spinor: packed -> canonical complex128. */
int tmqcd_unpack_spinor(const tmqcd_problem* prob, const void* in_packed, void* out_canon,
                        int prec, int subset, int nrhs, void* stream);

/* ---- the operator ------------------------------------------------------------ */
/* out = op(in) for nrhs packed fields of precision prec (in and out: the subset
 * the op acts on - odd input/even output for DSLASH_EO, even/odd for DSLASH_OE,
 * full for M*, even for MHAT*).  U_packed must be packed with (prec, recon).
 * out must not overlap in.  nrhs in [1, 16]; nrhs > 1 reuses each link load
 * across the right-hand sides. */
int tmqcd_dslash(const tmqcd_problem* prob, const void* U_packed, const void* in, void* out,
                 int op, int prec, int recon, int nrhs, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops that forbid hipMalloc): tmqcd_dslash with the operator's
 * temporaries (the odd half fields of MHAT, MHATDAG and MHATDAGMHAT, the full
 * field of MDAGM; nrhs * tmqcd_workspace_bytes(prob, op, 1 << prec, 1) bytes) in
 * a static device array of the library, TMQCD_NOALLOC_SCRATCH_BYTES (128 MiB) per
 * GPU, held from the library's load until the process ends.  Arguments, layouts,
 * results and errors are those of tmqcd_dslash (the same kernels, bitwise the same
 * output), minus ws; TMQCD_ESCRATCH when the temporaries do not fit (checked on
 * the host before any device call; e.g. MHATDAGMHAT in FP64 fits up to 24^3 x 48
 * with one right-hand side).  The call allocates nothing (no hipMalloc, hipFree
 * or allocating library routine); on its first call for a device it looks up
 * that device's address of the array (the device of `stream`, or the current
 * device for the null stream).  Every call on one GPU uses the same array: calls
 * that overlap in time on one GPU (different streams, or host threads) race on it
 * and must be ordered by the caller.  The operators without temporaries
 * (DSLASH_EO, DSLASH_OE, M, MDAG) do not touch it. */
#define TMQCD_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
size_t tmqcd_noalloc_scratch_bytes(void);
int tmqcd_dslash_noalloc(const tmqcd_problem* prob, const void* U_packed, const void* in, void* out, int op,
                         int prec, int recon, int nrhs, void* stream);

/* ---- the solver: CG on M^+M (full) or Mhat^+ Mhat (even sites) -------------- */
/* The paper's section 2.1: D phi = psi is solved with a Krylov method (CG or
 * BiCGStab) because D is a large sparse matrix whose matrix-vector product is
 * repeated at every iteration; CG needs a hermitian positive-definite operator,
 * here the normal operator M^+M, or Mhat^+Mhat of the even-odd Schur complement
 * (the same section's even-odd preconditioning).  Mixed precision (an FP32 or
 * FP16 inner operator inside an FP64 defect correction) is the mixed solver the
 * paper's conclusions (section 6) leave to future work. */
typedef struct {
    double  tol;             /* stop when ||b - A x||_2 / ||b||_2 <= tol, recomputed in FP64 */
    int32_t max_iter;        /* cap on (inner) CG iterations */
    int32_t op;              /* TMQCD_MDAGM or TMQCD_MHATDAGMHAT */
    int32_t inner_prec;      /* TMQCD_F64: plain FP64 CG; TMQCD_F32 / TMQCD_F16: mixed precision */
    int32_t recon;           /* link storage of every U_packed[] given */
    double  reliable_delta;  /* mixed: reliable update when the residual fell by this factor
                                (0 -> 1e-4 for FP32, 1e-2 for FP16 inner precision) */
    int32_t check_every;     /* most iterations queued between host residual checks (0 -> 32); batches
                                are sized from the observed convergence rate */
    int32_t x_is_zero;       /* 1: ignore the contents of x and start from x0 = 0 */
    int32_t use_graph;       /* tmqcd_cg: 1 replays the iterations from a hipGraph of 8 iterations
                                captured once per solve (saves host launch time, a few us per
                                iteration on lattices up to 8^3 x 16, for the cost of one capture per
                                solve: worth it for long solves on small lattices); 0 or -1 launch
                                every iteration.  Results are bitwise those of the eager launches.
                                With 1 on the null stream the solve runs on a blocking stream of its
                                own. */
    int32_t nrhs;            /* tmqcd_cg: right-hand sides solved together (0 or 1: one; up to 16).
                                With nrhs > 1 (FP64 only: inner_prec = TMQCD_F64, use_graph 0 or -1)
                                b and x hold nrhs packed fields one after the other, stats points at
                                nrhs structs, and every operator application is one multi-RHS launch
                                reading each link once for all columns; each column has its own FP64
                                scalars, residuals and stop test (the paper's section 2.1: a
                                propagator needs one inversion per spin-colour source). */
} tmqcd_cg_opts;

typedef struct {
    int32_t iters;             /* CG iterations, all precisions */
    int32_t reliable_updates;  /* outer cycles: FP64 true-residual recomputations that ended an inner
                                  cycle (the last one confirms convergence) */
    int32_t converged;         /* 1 if the true residual met tol */
    int32_t hop_launches;      /* hop kernels launched (for bandwidth accounting; with nrhs > 1 the
                                  multi-RHS launches, shared by the columns) */
    double  true_rel_residual; /* ||b - A x|| / ||b|| in FP64 at exit */
    double  iter_rel_residual; /* recursively updated residual at exit */
    double  seconds;           /* host wall time of the call */
    int32_t inner_iters;       /* iterations whose operator ran in the inner (FP32 / FP16) precision:
                                  iters for a mixed solve, 0 for FP64 */
    int32_t reserved;          /* 0 */
} tmqcd_cg_stats;

/* Solve A x = b, A = op (the paper's section 2.1, CG on the normal operator).
 * b and x are packed FP64 fields (full for MDAGM, even for MHATDAGMHAT; opts->nrhs
 * of them one after the other for the multi-RHS solve); x may not overlap b.
 * U_packed[p] is the gauge field packed at precision p (index TMQCD_F64/F32/F16)
 * with opts->recon; U_packed[TMQCD_F64] is always required, U_packed[inner_prec]
 * for mixed precision; unused entries may be NULL.  Mixed precision runs the inner
 * CG with FP32 or FP16 Dslash storage and FP64 reductions, and restarts it with an
 * FP64 residual b - A x whenever the iterated residual dropped by reliable_delta
 * (defect correction with reliable updates).  stats: host memory, one struct (nrhs
 * structs for nrhs > 1).  ws: tmqcd_workspace_bytes(prob, op, 1 | 1 << inner_prec,
 * nrhs) bytes of device memory, 256-byte aligned, overlapping neither b nor x.
 * Returns TMQCD_ENOCONV if max_iter was reached (x holds the last iterate),
 * TMQCD_EBREAKDOWN on a non-finite residual or p^+ A p <= 0 (for nrhs > 1: in some
 * column; the other columns are solved), TMQCD_EINVAL / EALIGN / EALIAS /
 * EWORKSPACE on bad arguments (checked before any device call), TMQCD_EHIP if a
 * HIP call failed. */
int tmqcd_cg(const tmqcd_problem* prob, const void* const U_packed[3], const void* b, void* x,
             const tmqcd_cg_opts* opts, tmqcd_cg_stats* stats, void* ws, size_t ws_bytes,
             void* stream);

/* BiCGStab (the paper's other Krylov solver for D phi = psi, its §2.1; van der
 * Vorst's algorithm) on the non-hermitian operator itself: opts->op = TMQCD_M
 * (b, x full fields) or TMQCD_MHAT (the even-odd Schur complement; b, x even
 * fields), FP64 only (opts->inner_prec must be TMQCD_F64), links U_packed FP64
 * with opts->recon.  Stops when the true residual ||b - A x|| / ||b|| <= tol
 * (recomputed in FP64 when the recursive one got there; the recursion restarts
 * from the true residual otherwise, counted in stats->reliable_updates).
 * opts->reliable_delta is ignored; check_every and x_is_zero act as for CG.
 * stats->iters counts BiCGStab iterations (two operator applications each).
 * ws: tmqcd_bicgstab_workspace_bytes(prob, op) bytes, device, 256-byte
 * aligned, caller-owned; x may not overlap b; ws overlaps none of b, x, U_packed.
 * Returns TMQCD_ENOCONV at max_iter, TMQCD_EBREAKDOWN on (rt, v) = 0, omega = 0
 * or a non-finite residual, else the errors of tmqcd_cg. */
size_t tmqcd_bicgstab_workspace_bytes(const tmqcd_problem* prob, int op);
int tmqcd_bicgstab(const tmqcd_problem* prob, const void* U_packed, const void* b, void* x,
                   const tmqcd_cg_opts* opts, tmqcd_cg_stats* stats, void* ws, size_t ws_bytes, void* stream);

/* ---- several lattices at once ------------------------------------------------ */
/* The paper's section 2.1 notes that thermal lattices (small temporal extent)
 * are simulated with less parallelism and need many parameter values and high
 * statistics: several such lattices are solved together here.
 * FP64 CG on Mhat^+ Mhat for n (1..8) lattices of any volumes in one solve:
 * every stage of an iteration is a single grid-stride launch over the tiles of
 * all lattices (each with its own solver state; converged lattices are skipped),
 * and with use_graph = 1 one iteration is captured once in a hipGraph and
 * replayed between host checks (on the null stream the library captures on a
 * stream of its own).  probs[n], U_packed[n] (FP64, opts->recon), b[n], x[n]
 * (packed FP64 even fields; x may not overlap any b or another x), stats[n].
 * opts->op must be TMQCD_MHATDAGMHAT and opts->inner_prec TMQCD_F64; x starts
 * from 0.  Results equal those of tmqcd_cg on each lattice alone.
 * Returns TMQCD_ENOCONV if a lattice hit max_iter (the others are solved). */
size_t tmqcd_cg_batch_workspace_bytes(int n, const tmqcd_problem* probs);
int tmqcd_cg_batch(int n, const tmqcd_problem* probs, const void* const* U_packed, const void* const* b,
                   void* const* x, const tmqcd_cg_opts* opts, tmqcd_cg_stats* stats, int use_graph,
                   void* ws, size_t ws_bytes, void* stream);

/* ---- the fermion force -------------------------------------------------------- */
/* The gradient G^a_mu(x) = dS_f/dw^a of S_f = phi^+ (M^+ M)^{-1} phi with respect
 * to U_mu(x) -> exp(i w^a T^a) U_mu(x), T^a = lambda^a / 2, given X = (M^+ M)^{-1} phi
 * and Y = M X as packed FP64 full fields (the paper's section 2.2, the fermion
 * force: the derivative of D^{-1} needs one inversion, and only the hopping part
 * of M depends on U):
 *   G^a = -2 kappa Im Tr[T^a (b+ Q1 - conj(b+) Q2)],
 *   Q1 = sum_spin [(1 - gamma_mu) U_mu(x) X(x+mu)] (x) Y(x)^+,
 *   Q2 = sum_spin X(x) (x) [U_mu(x) (1 + gamma_mu) Y(x+mu)]^+.
 * Y = NULL: the call computes Y = M X itself, into ws (tmqcd_force_workspace_bytes
 * bytes: one packed FP64 full field; device, 256-byte aligned, caller-owned,
 * overwritten); with Y given, ws may be NULL.
 * dSdw[V][4][8] (device, float64, canonical) receives scale * G (accumulate = 0)
 * or has scale * G added (accumulate = 1): with dSdw = p and scale = -dt this is
 * the HMC momentum update.  U_packed: FP64 with the given recon.
 * Errors: TMQCD_EINVAL (bad problem or recon, X or dSdw NULL, non-finite scale,
 * accumulate not 0/1), TMQCD_EALIGN, TMQCD_EWORKSPACE (Y NULL and ws missing or
 * short), TMQCD_EALIAS (dSdw overlaps X, Y, U_packed or ws; ws overlaps X or
 * U_packed); TMQCD_EHIP if a launch fails. */
size_t tmqcd_force_workspace_bytes(const tmqcd_problem* prob);
int tmqcd_force(const tmqcd_problem* prob, const void* U_packed, int recon, const void* X, const void* Y,
                double* dSdw, double scale, int accumulate, void* ws, size_t ws_bytes, void* stream);

/* The force of the even-odd pseudofermion action S_f = phi_e^+ (Mhat^+ Mhat)^{-1} phi_e
 * (the paper's force section for the Schur complement of its even-odd
 * preconditioning; the hybrid Monte-Carlo of its ensemble-generation section runs
 * on this action), given X_e = (Mhat^+ Mhat)^{-1} phi_e as a packed FP64 even
 * field.  The links enter only through H_eo and H_oe, so G is the full-lattice
 * formula of tmqcd_force evaluated at
 *   X = (X_e, A(mu)^{-1} H_oe X_e),   Y = kappa (Y_e, A(-mu)^{-1} (H^+)_oe Y_e),  Y_e = Mhat X_e.
 * Three hops build X_o, Y_e and Y_o in ws (tmqcd_force_eo_workspace_bytes(prob)
 * bytes, device, 256-byte aligned, caller-owned, overwritten), then the force
 * kernel writes or accumulates scale * G into dSdw[V][4][8] as tmqcd_force does.
 * U_packed: FP64 with the given recon (any of the four encodings).  dSdw may not overlap X_e, U_packed or ws.
 * Errors: TMQCD_EINVAL (bad problem, recon, null pointer, non-finite scale,
 * accumulate not 0/1), TMQCD_EALIGN, TMQCD_EWORKSPACE (ws missing or short),
 * TMQCD_EALIAS; TMQCD_EHIP if a launch fails. */
size_t tmqcd_force_eo_workspace_bytes(const tmqcd_problem* prob);
int tmqcd_force_eo(const tmqcd_problem* prob, const void* U_packed, int recon, const void* X_e, double* dSdw,
                   double scale, int accumulate, void* ws, size_t ws_bytes, void* stream);

/* ---- hybrid Monte-Carlo helpers (the paper's ensemble-generation section) ----- */
/* Gradient of the Wilson plaquette action S_g = (beta/3) sum_{x,mu<nu} (3 - Re Tr P_mu_nu(x))
 * (the paper's tree-level Symanzik action at c1 = 0; no boundary phases):
 * G^a = (beta/3) Im Tr[T^a U_mu(x) V_mu(x)], V_mu the six staples.  Written or
 * accumulated into dSdw[V][4][8] like tmqcd_force.  U_packed: FP64, RECON18. */
int tmqcd_gauge_force(const tmqcd_problem* prob, const void* U_packed, double beta, double* dSdw,
                      double scale, int accumulate, void* stream);
/* Gradient of the paper's tree-level Symanzik gauge action (its gauge-sector
 * equation; the force splits into plaquette and rectangle parts as in its HMC
 * section):
 *   S_g = (beta/3) sum_x [ c0 sum_{mu<nu} (3 - Re Tr P_mu_nu(x)) + c1 sum_{mu!=nu} (3 - Re Tr R_mu_nu(x)) ],
 * c0 = 1 - 8 c1, R_mu_nu(x) the rectangle two links long in mu and one in nu
 * (each geometric rectangle counted once).  Tree-level improvement takes
 * c1 = -1/12; c1 = 0 gives tmqcd_gauge_force's Wilson action.
 *   G^a = (beta/3) Im Tr[T^a U_mu(x) V_mu(x)],  V_mu = c0 (6 plaquette staples) + c1 (18 rectangle staples),
 * written or accumulated into dSdw[V][4][8] like tmqcd_force.  U_packed: FP64, RECON18.
 * For c1 != 0 a first kernel stores the 24 single plaquette staples of every
 * site in ws (tmqcd_gauge_force_tlsym_workspace_bytes(prob) bytes, 3456 per
 * site: device, 256-byte aligned, caller-owned, overwritten) and each rectangle
 * staple is then a product of two stored staples and a link (U^+ U = 1); for
 * c1 = 0 ws is not used and may be NULL.
 * Errors: TMQCD_EINVAL (bad problem, null pointer, non-finite beta, c1 or scale,
 * accumulate not 0/1), TMQCD_EALIGN, TMQCD_EWORKSPACE (c1 != 0 and ws missing
 * or short), TMQCD_EALIAS (dSdw overlaps U_packed; ws overlaps U_packed or dSdw). */
size_t tmqcd_gauge_force_tlsym_workspace_bytes(const tmqcd_problem* prob);
int tmqcd_gauge_force_tlsym(const tmqcd_problem* prob, const void* U_packed, double beta, double c1, double* dSdw,
                            double scale, int accumulate, void* ws, size_t ws_bytes, void* stream);
/* U_mu(x) <- exp(i dt p^a T^a) U_mu(x) for every link, in place on the packed
 * FP64 RECON18 field; p[V][4][8] (device, float64).  The exponential is exact to
 * FP64 rounding (Taylor polynomial after scaling, then squaring). */
int tmqcd_update_links(const tmqcd_problem* prob, void* U_packed, const double* p, double dt,
                       void* stream);
/* ---- pure-gauge updates (the paper's heatbath section) ---------------------- */
/* One sweep over all links of the Wilson plaquette action
 * S = (beta/3) sum (3 - Re Tr P), in place on the packed RECON18 links of
 * precision prec (TMQCD_F64, or TMQCD_F32 with FP32 arithmetic, the precision
 * in which the paper measures its heatbath):
 * direction by direction and parity by parity (8 launches; the links of one
 * direction and parity do not appear in each other's staples), each link
 * updated through the SU(2) subgroups (0,1), (0,2), (1,2) (Cabibbo-Marinari).
 *   tmqcd_heatbath:  the exact SU(2) heatbath in each subgroup (Creutz's
 *                    inversion below alpha = 2, Kennedy-Pendleton above);
 *                    random numbers from the counter-based Philox4x32-10 with
 *                    key `seed` and counter (4 s + mu, sweep, subgroup * 2^16 +
 *                    trial, 0), s the canonical site index, so a sweep is a
 *                    pure function of (links, beta, seed, sweep).
 *   tmqcd_overrelax: the microcanonical reflection r = (s^+)^2 in each
 *                    subgroup (no random numbers; keeps the action).
 * Errors: TMQCD_EINVAL (bad problem, null links, prec not FP64/FP32, beta
 * negative or not finite, more than 2^32 links), TMQCD_EALIGN; TMQCD_EHIP if a
 * launch fails. */
int tmqcd_heatbath(const tmqcd_problem* prob, void* U_packed, int prec, double beta, uint64_t seed, uint32_t sweep,
                   void* stream);
int tmqcd_overrelax(const tmqcd_problem* prob, void* U_packed, int prec, void* stream);

/* The change of the HMC Hamiltonian H = 1/2 sum p^2 + S_g + S_f (the paper's section
 * 2.2: the Metropolis step accepts with min(1, exp(-(H' - H)))) between the states
 * (U0, p0, X0) and (U1, p1, X1), summed site by site in FP64 so that no difference of
 * two large totals is formed:
 *   dH = sum_x [ 1/2 sum_{mu,a} (p1^2 - p0^2)
 *               + (beta/3) (c0 sum_{mu<nu} Re Tr(P0 - P1) + c1 sum_{mu!=nu} Re Tr(R0 - R1))
 *               + Re phi(x)^+ (X1(x) - X0(x)) ],   c0 = 1 - 8 c1,
 * the gauge action of tmqcd_gauge_force_tlsym (c1 = 0: Wilson; beta = 0: none) and
 * S_f = Re phi^+ X with X the solution of the pseudofermion's system at each state
 * (X = (M^+M)^{-1} phi for subset TMQCD_FULL, (Mhat^+Mhat)^{-1} phi_e for TMQCD_EVEN).
 * U0, U1: packed FP64 RECON18 links; p0, p1: double[V][4][8]; phi, X0, X1: packed FP64
 * fields of `subset`.  result[0..3] (device): dH and its kinetic, gauge and
 * fermion parts.  ws: tmqcd_workspace_bytes(prob, -1, 1, 1) bytes.
 * Errors: TMQCD_EINVAL (bad problem, null pointer, subset not FULL/EVEN, non-finite
 * beta or c1), TMQCD_EALIGN, TMQCD_EWORKSPACE, TMQCD_EALIAS (ws or result overlapping
 * an input); TMQCD_EHIP if a launch fails. */
int tmqcd_delta_h(const tmqcd_problem* prob, const void* U0, const void* U1, const double* p0, const double* p1,
                  const void* phi, const void* X0, const void* X1, int subset, double beta, double c1,
                  double* result, void* ws, size_t ws_bytes, void* stream);

/* Deterministic FP64 reductions into device memory.  ws: tmqcd_workspace_bytes(prob, -1, 1, 1) bytes.
 *   tmqcd_plaquette:      result[0] = sum_{x, mu<nu} Re Tr P_mu_nu(x)       (U_packed FP64 RECON18)
 *   tmqcd_rectangle:      result[0] = sum_{x, mu!=nu} Re Tr R_mu_nu(x)      (the 12 V rectangles of
 *                         tmqcd_gauge_force_tlsym; U_packed FP64 RECON18)
 *   tmqcd_momentum_norm2: result[0] = sum p^2 over all V*4*8 entries
 *   tmqcd_dot:            result[0] + i result[1] = x^+ y for packed FP64 fields of `subset` */
int tmqcd_plaquette(const tmqcd_problem* prob, const void* U_packed, double* result, void* ws,
                    size_t ws_bytes, void* stream);
int tmqcd_rectangle(const tmqcd_problem* prob, const void* U_packed, double* result, void* ws,
                    size_t ws_bytes, void* stream);
int tmqcd_momentum_norm2(const tmqcd_problem* prob, const double* p, double* result, void* ws,
                         size_t ws_bytes, void* stream);
int tmqcd_dot(const tmqcd_problem* prob, const void* x, const void* y, int subset, double* result,
              void* ws, size_t ws_bytes, void* stream);

/* ---- autotuning --------------------------------------------------------------- */
/* The paper tuned its kernels per GPU (its implementation-strategy section 4:
 * memory stride, lattice extents compiled in); here the launch shape of each hop kernel class is chosen by timing on
 * the caller's problem.  A shape is a block size (128 or 256 threads) and a
 * block order, i.e. which output sites a block covers:
 *   0  linear: block b covers half sites [b*w, b*w + w) of its parity;
 *   1  linear, block index remapped so that each XCD gets a contiguous range;
 *   2  every t-slice cut into 8 site ranges, one per XCD, each XCD walking
 *      through t (its t-neighbours are in slices it has in flight);
 *   3  the (y, z) plane cut into square regions sized to the L2, each XCD
 *      sweeping its regions one by one through all t;
 *   4  the lattice cut into 4 z-ranges (runs of z-planes) x 2 t-ranges, one
 *      block of them per XCD, each XCD walking through its t-range;
 *   5  as 4 with 2 z-ranges x 4 t-ranges.
 * Kernel classes: 0 hop (+ twisted-mass own term), 1 hop + |out|^2 (CG),
 * 2 hop + CG update, 3 multi-RHS hop (256 threads: 64 sites x 4 waves; the
 * order and the number of right-hand sides a block serves are tuned: with
 * fewer per block the lattice is swept once per group, the links are read once
 * per group, and fewer fields compete for the L2).  Only shapes whose output is bitwise identical to the
 * default shape's (256 threads; order 1, or 2 for class 3) are admitted (for classes 1 and 2
 * the reduction may differ by 1e-12 relative: the partial sums group
 * differently).  The fastest shape is recorded in a process-wide table keyed by
 * (GPU architecture, class, prec, recon, extents, nrhs) that later
 * tmqcd_dslash / tmqcd_cg / tmqcd_cg_batch calls on the same key use; keys
 * without an entry take the default shape.  The tuning calls synchronise the
 * stream. */
typedef struct {
    int32_t kernel_class;  /* 0..3 as above */
    int32_t block;         /* chosen threads per block */
    int32_t order;         /* chosen block order, 0..5 as above */
    int32_t group;         /* class 3: right-hand sides per block (0: all of them); else 0 */
    int32_t candidates;    /* shapes tried */
    int32_t rejected;      /* shapes whose output differed from the default's */
    double  us;            /* time per launch of the chosen shape */
    double  default_us;    /* time per launch of the default shape */
} tmqcd_tune_result;
/* Classes 0, 1, 2 (12 shapes each).  ws: at least tmqcd_tune_workspace_bytes. */
size_t tmqcd_tune_workspace_bytes(const tmqcd_problem* prob, int prec);
int tmqcd_tune(const tmqcd_problem* prob, const void* U_packed, int prec, int recon, void* ws,
               size_t ws_bytes, tmqcd_tune_result results[3], void* stream);
/* Class 3 for nrhs in [2, 16] (6 orders x groups of all, about half and
 * about a third of the right-hand sides).  ws: at least
 * tmqcd_tune_mrhs_workspace_bytes(prob, prec, nrhs) bytes. */
size_t tmqcd_tune_mrhs_workspace_bytes(const tmqcd_problem* prob, int prec, int nrhs);
int tmqcd_tune_mrhs(const tmqcd_problem* prob, const void* U_packed, int prec, int recon, int nrhs, void* ws,
                    size_t ws_bytes, tmqcd_tune_result* result, void* stream);
/* The table as JSON lines (one object per key).  Loading replaces the table and
 * fails with TMQCD_EINVAL on a malformed file or one tuned on another
 * architecture. */
int tmqcd_tune_save(const char* path);
int tmqcd_tune_load(const char* path);
void tmqcd_tune_clear(void);
/* Pins the shape of one class for this problem, precision and link
 * compression, as a tuning run would: classes 0..2 take nrhs = 1, block 128
 * or 256 and group 0; class 3 takes nrhs in [2, 16], block 256 and group in
 * [0, nrhs]; order 0..5.  TMQCD_EINVAL for any other value.  Host only. */
int tmqcd_tune_set(const tmqcd_problem* prob, int prec, int recon, int kernel_class, int nrhs, int block,
                   int order, int group);

/* ---- diagnostics ------------------------------------------------------------- */
/* Bandwidth probe (a measurement aid, not part of the method): with dst ==
 * NULL, reads `bytes` of src with 16-byte loads and xors every 32-bit word
 * into *xor_out (a device word the caller sets beforehand; required then);
 * otherwise copies src to dst (xor_out unused).  `grid` blocks of 256 threads
 * stride over the buffer; stream-ordered.  bytes must be a positive multiple
 * of 16, grid in [1, 65536], src and dst 16-byte aligned, xor_out 4-byte
 * aligned, no two of them overlapping. */
int tmqcd_hbm_probe(const void* src, void* dst, size_t bytes, int grid, uint32_t* xor_out, void* stream);

const char* tmqcd_error_string(int code);
int tmqcd_last_hip_error(void);   /* hipError_t of the last failed HIP call in this thread */

#ifdef __cplusplus
}
#endif
#endif /* TMQCD_H */
