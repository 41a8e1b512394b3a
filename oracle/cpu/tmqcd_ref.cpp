// Plain FP64 C++/OpenMP oracle of the twisted-mass Wilson operator, its even-odd
// Schur complement and CG (the second oracle: the same definitions as the NumPy
// oracle in oracle/dirac.py, written as loops over sites so that it runs at
// full lattice sizes on the host cores).
//
// TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the tests, the smoke check and the
// CPU-baseline leg of the benchmark load this library.  It shares no code, header,
// table or constant with the HIP library.
//
// Definitions (Bach, Lindenstruth, Philipsen, Pinke, "Lattice QCD based on
// OpenCL", section 2.1, the equation of D_tm and the even-odd paragraph), with
// the readings of the NumPy oracle:
//   M = A - kappa H,  A = 1 + i w gamma5,  w = 2 kappa mu  (hopping prefactor kappa);
//   (H psi)(x) = sum_mu [ b+_mu(x) (1 - gamma_mu) U_mu(x) psi(x + mu)
//                       + b-_mu(x) (1 + gamma_mu) U_mu(x - mu)^+ psi(x - mu) ],
//   b+_mu(x) = bc_mu on the hop that crosses the last slice, b-_mu(x) = conj(bc_mu)
//   on the one that crosses the first, 1 otherwise;
//   H^+ is H with gamma_mu -> -gamma_mu, A^+ = 1 - i w gamma5;
//   Mhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe on even sites,
//   Mhat^+ = A^+_ee - kappa^2 (H^+)_eo (A^+_oo)^{-1} (H^+)_oe.
// Gamma matrices: chiral basis gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]
// (k = x, y, z), gamma_t = [[0, -1], [-1, 0]], gamma5 = gamma_x gamma_y gamma_z gamma_t.
// Fields are canonical complex128 arrays: psi[V][4][3] (full) or [V/2][4][3] for
// one parity indexed by h = s >> 1, U[V][4][3][3] (U_mu(s), row-major); site
// s = x + Lx (y + Ly (z + Lz t)).
//
// CG is Hestenes-Stiefel from x0 = 0, stopping when the recursively updated
// residual satisfies |r| <= tol |b|; the true residual |b - A x| / |b| is
// recomputed at exit.  Reductions use OpenMP's sum reduction (FP64).
#include <omp.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

typedef std::complex<double> cd;

cd G[5][4][4];   // gamma_x, gamma_y, gamma_z, gamma_t, gamma5

void init_gammas() {
    static bool done = false;
    if (done) return;
    const cd I(0, 1);
    const cd sigma[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    for (int m = 0; m < 5; ++m)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) G[m][a][b] = 0;
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                G[k][a][2 + b] = -I * sigma[k][a][b];
                G[k][2 + a][b] = I * sigma[k][a][b];
            }
    for (int a = 0; a < 2; ++a) {
        G[3][a][2 + a] = -1;
        G[3][2 + a][a] = -1;
    }
    // gamma5 = gamma_x gamma_y gamma_z gamma_t as a matrix product
    cd t1[4][4], t2[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            t1[a][b] = 0;
            for (int c = 0; c < 4; ++c) t1[a][b] += G[0][a][c] * G[1][c][b];
        }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            t2[a][b] = 0;
            for (int c = 0; c < 4; ++c) t2[a][b] += t1[a][c] * G[2][c][b];
        }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            G[4][a][b] = 0;
            for (int c = 0; c < 4; ++c) G[4][a][b] += t2[a][c] * G[3][c][b];
        }
    done = true;
}

struct Lat {
    int L[4];
    int64_t V;
    double kappa, w;
    cd bc[4];
    const cd* U;
};

Lat make_lat(const int dims[4], double kappa, double mu, const double* bc, const double* U) {
    Lat l;
    l.V = 1;
    for (int i = 0; i < 4; ++i) {
        l.L[i] = dims[i];
        l.V *= dims[i];
        l.bc[i] = cd(bc[2 * i], bc[2 * i + 1]);
    }
    l.kappa = kappa;
    l.w = 2.0 * kappa * mu;
    l.U = reinterpret_cast<const cd*>(U);
    return l;
}

void coords_of(const Lat& l, int64_t s, int c[4]) {
    c[0] = (int)(s % l.L[0]);
    c[1] = (int)((s / l.L[0]) % l.L[1]);
    c[2] = (int)((s / ((int64_t)l.L[0] * l.L[1])) % l.L[2]);
    c[3] = (int)(s / ((int64_t)l.L[0] * l.L[1] * l.L[2]));
}
int64_t site_of(const Lat& l, const int c[4]) { return c[0] + l.L[0] * (c[1] + (int64_t)l.L[1] * (c[2] + (int64_t)l.L[2] * c[3])); }

// A field: full (index s) or one parity (index s >> 1).
struct Field {
    cd* p;
    bool half;
    cd* at(int64_t s) const { return p + 12 * (half ? (s >> 1) : s); }
};

// out(s) = sum over the eight terms, for every site s of parity out_par (-1: all sites);
// sgn = +1 for H, -1 for H^+.  in must hold the neighbours (the other parity at least).
void hop(const Lat& l, Field in, Field out, int out_par, double sgn) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < l.V; ++s) {
        int c[4];
        coords_of(l, s, c);
        const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
        if (out_par >= 0 && par != out_par) continue;
        cd acc[4][3];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 3; ++b) acc[a][b] = 0;
        for (int mu = 0; mu < 4; ++mu) {
            int cf[4], cb[4];
            for (int i = 0; i < 4; ++i) cf[i] = cb[i] = c[i];
            cf[mu] = (c[mu] + 1) % l.L[mu];
            cb[mu] = (c[mu] + l.L[mu] - 1) % l.L[mu];
            const int64_t sf = site_of(l, cf), sb = site_of(l, cb);
            const cd phf = c[mu] == l.L[mu] - 1 ? l.bc[mu] : cd(1, 0);
            const cd phb = c[mu] == 0 ? std::conj(l.bc[mu]) : cd(1, 0);
            const cd* uf = l.U + 9 * (4 * s + mu);    // U_mu(x)
            const cd* ub = l.U + 9 * (4 * sb + mu);   // U_mu(x - mu)
            const cd* pf = in.at(sf);
            const cd* pb = in.at(sb);
            // colour: t = U psi(x + mu), v = U^+ psi(x - mu), per spin
            cd t[4][3], v[4][3];
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    t[sp][a] = 0;
                    v[sp][a] = 0;
                    for (int b = 0; b < 3; ++b) {
                        t[sp][a] += uf[3 * a + b] * pf[3 * sp + b];
                        v[sp][a] += std::conj(ub[3 * b + a]) * pb[3 * sp + b];
                    }
                }
            // spin: (1 - sgn gamma_mu) t and (1 + sgn gamma_mu) v
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cd f = t[sp][a], g = v[sp][a];
                    for (int q = 0; q < 4; ++q) {
                        f -= sgn * G[mu][sp][q] * t[q][a];
                        g += sgn * G[mu][sp][q] * v[q][a];
                    }
                    acc[sp][a] += phf * f + phb * g;
                }
        }
        cd* o = out.at(s);
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) o[3 * sp + a] = acc[sp][a];
    }
}

// out = c_own (1 + i wsgn gamma5)^(inv ? -1 : 1) own + c_hop * hopped, per site of `n` sites
// (the twisted diagonal is diagonal in spin in the chiral basis, but it is applied
// here as the spin matrix 1 + i w gamma5, or its inverse (1 - i w gamma5) / (1 + w^2)).
void twist_combine(const Lat& l, int64_t n, const cd* own, double wsgn, bool inv, cd c_hop, const cd* hopped,
                   cd* out) {
    const cd I(0, 1);
    cd A[4][4];
    const double w = wsgn * l.w;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const cd id = a == b ? 1.0 : 0.0;
            A[a][b] = inv ? (id - I * w * G[4][a][b]) / (1.0 + w * w) : id + I * w * G[4][a][b];
        }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const cd* x = own + 12 * i;
        cd* o = out + 12 * i;
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                cd v = 0;
                for (int q = 0; q < 4; ++q) v += A[sp][q] * x[3 * q + a];
                o[3 * sp + a] = v + (hopped ? c_hop * hopped[12 * i + 3 * sp + a] : cd(0, 0));
            }
    }
}

enum Op { kHop = 0, kM, kMdag, kMdagM, kMhat, kMhatdag, kMhatdagMhat, kHopEO, kHopOE };

bool full_op(int op) { return op == kHop || op == kM || op == kMdag || op == kMdagM; }

// M psi or M^+ psi (full fields)
void apply_M(const Lat& l, const cd* in, cd* out, bool dag, std::vector<cd>& tmp) {
    tmp.resize(12 * l.V);
    hop(l, Field{const_cast<cd*>(in), false}, Field{tmp.data(), false}, -1, dag ? -1.0 : 1.0);
    twist_combine(l, l.V, in, dag ? -1.0 : 1.0, false, -l.kappa, tmp.data(), out);
}

// Mhat psi_e or Mhat^+ psi_e (even fields)
void apply_Mhat(const Lat& l, const cd* in, cd* out, bool dag, std::vector<cd>& t1, std::vector<cd>& t2) {
    const int64_t vh = l.V / 2;
    const double sgn = dag ? -1.0 : 1.0;
    t1.resize(12 * vh);
    t2.resize(12 * vh);
    hop(l, Field{const_cast<cd*>(in), true}, Field{t1.data(), true}, 1, sgn);     // H_oe in
    twist_combine(l, vh, t1.data(), sgn, true, 0.0, nullptr, t2.data());          // A_oo^{-1}
    hop(l, Field{t2.data(), true}, Field{t1.data(), true}, 0, sgn);               // H_eo
    twist_combine(l, vh, in, sgn, false, -l.kappa * l.kappa, t1.data(), out);
}

struct Work {
    std::vector<cd> a, b, c, d;
};

int64_t field_sites(const Lat& l, int op) { return full_op(op) ? l.V : l.V / 2; }

int apply(const Lat& l, int op, const cd* in, cd* out, Work& w) {
    const int64_t vh = l.V / 2;
    switch (op) {
        case kHop: hop(l, Field{const_cast<cd*>(in), false}, Field{out, false}, -1, 1.0); return 0;
        case kHopEO: hop(l, Field{const_cast<cd*>(in), true}, Field{out, true}, 0, 1.0); return 0;
        case kHopOE: hop(l, Field{const_cast<cd*>(in), true}, Field{out, true}, 1, 1.0); return 0;
        case kM: apply_M(l, in, out, false, w.a); return 0;
        case kMdag: apply_M(l, in, out, true, w.a); return 0;
        case kMdagM:
            w.b.resize(12 * l.V);
            apply_M(l, in, w.b.data(), false, w.a);
            apply_M(l, w.b.data(), out, true, w.a);
            return 0;
        case kMhat: apply_Mhat(l, in, out, false, w.a, w.b); return 0;
        case kMhatdag: apply_Mhat(l, in, out, true, w.a, w.b); return 0;
        case kMhatdagMhat:
            w.c.resize(12 * vh);
            apply_Mhat(l, in, w.c.data(), false, w.a, w.b);
            apply_Mhat(l, w.c.data(), out, true, w.a, w.b);
            return 0;
    }
    return -1;
}

double dot_re(const cd* a, const cd* b, int64_t n) {
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i) s += (std::conj(a[i]) * b[i]).real();
    return s;
}

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

// Threads used by the parallel loops (set with ref_set_threads or OMP_NUM_THREADS).
int ref_threads(void) { return omp_get_max_threads(); }
void ref_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}

// out = op(in); op: 0 H (full), 1 M, 2 M^+, 3 M^+M (full fields), 4 Mhat, 5 Mhat^+,
// 6 Mhat^+Mhat (even fields), 7 H_eo (odd in, even out), 8 H_oe (even in, odd out).
// bc: (re, im) per direction.  Returns 0, or -1 for an unknown op or odd extents.
int ref_apply(int op, const int* dims, double kappa, double mu, const double* bc, const double* U, const double* in,
              double* out) {
    init_gammas();
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 2 || dims[i] % 2) return -1;
    const Lat l = make_lat(dims, kappa, mu, bc, U);
    Work w;
    return apply(l, op, reinterpret_cast<const cd*>(in), reinterpret_cast<cd*>(out), w);
}

// ||b - op x|| / ||b|| in FP64.
double ref_true_rel_residual(int op, const int* dims, double kappa, double mu, const double* bc, const double* U,
                             const double* b, const double* x) {
    init_gammas();
    const Lat l = make_lat(dims, kappa, mu, bc, U);
    const int64_t n = 12 * field_sites(l, op);
    std::vector<cd> ax(n);
    Work w;
    if (apply(l, op, reinterpret_cast<const cd*>(x), ax.data(), w) != 0) return NAN;
    const cd* bb = reinterpret_cast<const cd*>(b);
    double rr = 0, nb = 0;
#pragma omp parallel for reduction(+ : rr, nb) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        rr += std::norm(bb[i] - ax[i]);
        nb += std::norm(bb[i]);
    }
    return std::sqrt(rr / nb);
}

// CG on op = 3 (M^+M, full fields) or 6 (Mhat^+Mhat, even fields) from x = 0 to
// |r| <= tol |b| (recursive residual), at most max_iter iterations.  stats (host, 6
// doubles): iterations, true relative residual at exit, seconds, and the iteration
// count, seconds and true relative residual of the iterate at which the recursive
// residual first reached report_tol (the same solve to a looser tolerance; the true
// residual of that iterate is computed outside the timed region).  Returns 0, 1 if
// max_iter was reached, -1 on bad arguments, -2 on breakdown.
int ref_cg(int op, const int* dims, double kappa, double mu, const double* bc, const double* U, const double* b,
           double* x, double tol, int max_iter, double report_tol, double* stats) {
    init_gammas();
    if (op != kMdagM && op != kMhatdagMhat) return -1;
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 2 || dims[i] % 2) return -1;
    const Lat l = make_lat(dims, kappa, mu, bc, U);
    const int64_t n = 12 * field_sites(l, op);
    const cd* bv = reinterpret_cast<const cd*>(b);
    cd* xv = reinterpret_cast<cd*>(x);
    std::vector<cd> r(bv, bv + n), p(bv, bv + n), ap(n), x_report;
    Work w;
    for (int64_t i = 0; i < n; ++i) xv[i] = 0;
    const double t0 = now();
    const double bb = dot_re(bv, bv, n);
    double rr = bb;
    int k = 0, k_rep = -1;
    double t_rep = 0;
    int rc = 0;
    while (rr > tol * tol * bb) {
        if (k_rep < 0 && rr <= report_tol * report_tol * bb) {
            k_rep = k;
            t_rep = now() - t0;
            x_report.assign(xv, xv + n);
        }
        if (k >= max_iter) {
            rc = 1;
            break;
        }
        apply(l, op, p.data(), ap.data(), w);
        const double pap = dot_re(p.data(), ap.data(), n);
        if (!(pap > 0)) {
            rc = -2;
            break;
        }
        const double alpha = rr / pap;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            xv[i] += alpha * p[i];
            r[i] -= alpha * ap[i];
        }
        const double rr_new = dot_re(r.data(), r.data(), n);
        const double beta = rr_new / rr;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        ++k;
    }
    if (k_rep < 0) {   // the looser tolerance was met together with tol
        k_rep = k;
        t_rep = now() - t0;
        x_report.assign(xv, xv + n);
    }
    const double secs = now() - t0;
    stats[0] = k;
    stats[1] = ref_true_rel_residual(op, dims, kappa, mu, bc, U, b, x);
    stats[2] = secs;
    stats[3] = k_rep;
    stats[4] = t_rep;
    stats[5] = ref_true_rel_residual(op, dims, kappa, mu, bc, U, b, reinterpret_cast<const double*>(x_report.data()));
    return rc;
}

}  // extern "C"
