// Fermion force: the gradient of S_f = phi^+ (M^+ M)^{-1} phi with respect to
// the eight su(3) directions of every link (paper: the HMC force section; the
// derivative of D^{-1} needs one inversion, and only the hopping part of the
// twisted-mass matrix depends on U).
//
// With X = (M^+ M)^{-1} phi and Y = M X, dS_f = 2 kappa Re(Y^+ dH X), which per
// link U_mu(x) -> exp(i w^a T^a) U_mu(x) gives
//   G^a = -2 kappa Im Tr[T^a (b+ Q1 - conj(b+) Q2)]
//   Q1 = sum_spin [(1 - gamma_mu) U X(x+mu)] (x) Y(x)^+
//   Q2 = sum_spin X(x) (x) [U (1 + gamma_mu) Y(x+mu)]^+
// One thread per (site, direction); each output is written once, so no
// atomics are needed.  The spin projectors are applied as in the hop, and the
// rank-2 projectors halve the spin sums of Q1 and Q2 (see project below).
#include "device.h"
#include "internal.h"


namespace tmqcd {
namespace {

constexpr int kPerm[4][2] = {{1, 0}, {1, 0}, {0, 1}, {0, 1}};
constexpr int kB[4][2] = {{3, 3}, {2, 0}, {3, 1}, {2, 2}};
constexpr int kBd[4][2] = {{1, 1}, {0, 2}, {1, 3}, {2, 2}};

// The rows of (1 + eps gamma_mu) v: h = v_up + eps B v_dn (the lower two rows are
// eps B^+ h).  In the chiral basis (1 + eps gamma_mu) = R P with P = [1, eps B] and
// R^+ = P, so for any a, b:  sum_spin [(1 + eps gamma_mu) a] (x) b^+ = sum_{r=0,1} (P a)_r (x) (P b)_r^+,
// which halves the outer products of Q1 and Q2.
template <int MU, int EPS>
__device__ __forceinline__ void project(Half<double>& h, const Spinor<double>& v) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int src = 2 + kPerm[MU][r];
        const int code = (kB[MU][r] + (EPS > 0 ? 0 : 2)) & 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const C<double> z = v.s[src][c];
            C<double> bz;
            switch (code) {
                case 0: bz = z; break;
                case 1: bz = {-z.im, z.re}; break;
                case 2: bz = {-z.re, -z.im}; break;
                default: bz = {z.im, -z.re}; break;
            }
            h.s[r][c] = v.s[r][c] + bz;
        }
    }
}

// g = U h on both rows
__device__ __forceinline__ void umul(Half<double>& g, const Su3<double>& u, const Half<double>& h) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            g.s[r][a] = u.m[a][0] * h.s[r][0] + u.m[a][1] * h.s[r][1] + u.m[a][2] * h.s[r][2];
}

struct ForceK {
    const char* gauge;
    const char* X[2];   // by parity: the even and the odd half of X
    const char* Y[2];
    double* out;
    int64_t stride, gstride;
    int L[4];
    int lxh, vh;
    C<double> bc[4];
    double kappa;
    double scale;
    int accumulate;
    int slice, q, tq, lt;    // half sites per t-slice, per XCD range, blocks per range, L_t (force_block_site)
};

// The 64 sites of block bid and their parity.  Hardware blocks go round-robin over
// the 8 XCDs (block b on XCD b % 8).  Every t-slice is cut into 8 ranges of q half
// sites, range x belonging to XCD x, which walks its ranges slice by slice, the
// even and the odd block of the same 64 half sites in turn: the t-neighbours it
// reads are the next slice of its own range, loaded moments later as own sites,
// and X, Y of one parity are read as neighbours by the blocks of the other parity
// while still in the XCD's L2.  Against all even blocks followed by all odd ones
// in lattice order this measured 40.8 vs 42.6 us at 16^3 x 32, 212 us for both at
// 24^3 x 48 and 639 vs 683 us at 32^3 x 64 (one GPU, the two builds run alternately), with
// bitwise the same output; giving each XCD one contiguous eighth of the lattice
// instead lost on 32^3 x 64, whose t-slice of X and Y no longer fits in L2.  So did
// cutting each range along y into chunks walked through t one after the other
// (32^3 x 64: 17 % less fetched from HBM, 15 % slower), and giving each XCD one of 4
// (or 2) z-ranges of the slices of one of 2 (or 4) t-ranges (16^3 x 32: 2 % faster,
// 24^3 x 48: the same, 32^3 x 64: 2.5 % slower).
__device__ __forceinline__ bool force_block_site(const ForceK& a, int bid, int lane, int& par, int& h) {
    const int x = bid & (kNumXcd - 1), k = bid / kNumXcd;
    const int t = k / (2 * a.tq), rem = k - t * 2 * a.tq;
    par = rem & 1;
    const int first = x * a.q + (rem >> 1) * 64 + lane;
    const int end = min((x + 1) * a.q, a.slice);
    h = t * a.slice + first;
    return t < a.lt && first < end;
}

template <int R, int MU>
__device__ __forceinline__ void force_dir(const ForceK& a, int par, int h, int nh, bool cross, double* g) {
    // Q = b+ Q1 - conj(b+) Q2 with Q1 = sum_r [U P- X(x+mu)]_r (x) [P- Y(x)]_r^+ and
    // Q2 = sum_r [P+ X(x)]_r (x) [U P+ Y(x+mu)]_r^+, accumulated one term at a time:
    // each spinor is projected right after its load and each outer product added to Q
    // as soon as both of its half spinors exist, so few of them are live at once.
    const C<double> b = cross ? a.bc[MU] : C<double>{1.0, 0.0};
    Su3<double> u;
    LinkIO<TMQCD_F64, R>::template load<true>(u, a.gauge, a.gstride, par, MU, h);
    C<double> q[3][3];
    {
        Half<double> z, w;
        {
            Spinor<double> v;
            SpinorIO<TMQCD_F64>::load(v, a.Y[par], a.stride, h);
            project<MU, -1>(z, v);
        }
        {
            Spinor<double> v;
            Half<double> hh;
            SpinorIO<TMQCD_F64>::load(v, a.X[1 - par], a.stride, nh);
            project<MU, -1>(hh, v);
            umul(w, u, hh);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                C<double> q1 = {0, 0};
#pragma unroll
                for (int r = 0; r < 2; ++r) q1 = q1 + cmul_cj(z.s[r][j], w.s[r][i]);   // w_i conj(z_j)
                q[i][j] = b * q1;
            }
    }
    {
        Half<double> z, w;
        {
            Spinor<double> v;
            SpinorIO<TMQCD_F64>::load(v, a.X[par], a.stride, h);
            project<MU, +1>(z, v);
        }
        {
            Spinor<double> v;
            Half<double> hh;
            SpinorIO<TMQCD_F64>::load(v, a.Y[1 - par], a.stride, nh);
            project<MU, +1>(hh, v);
            umul(w, u, hh);
        }
        const C<double> bc = conj(b);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                C<double> q2 = {0, 0};
#pragma unroll
                for (int r = 0; r < 2; ++r) q2 = q2 + cmul_cj(w.s[r][j], z.s[r][i]);   // z_i conj(w_j)
                q[i][j] = q[i][j] - bc * q2;
            }
    }
    // Im Tr(lambda^a Q) for the eight Gell-Mann matrices
    const double k = -a.kappa;   // -2 kappa * (1/2) from T^a = lambda^a / 2
    g[0] = k * (q[1][0].im + q[0][1].im);
    g[1] = k * (q[0][1].re - q[1][0].re);
    g[2] = k * (q[0][0].im - q[1][1].im);
    g[3] = k * (q[2][0].im + q[0][2].im);
    g[4] = k * (q[0][2].re - q[2][0].re);
    g[5] = k * (q[2][1].im + q[1][2].im);
    g[6] = k * (q[1][2].re - q[2][1].re);
    g[7] = k * (q[0][0].im + q[1][1].im - 2.0 * q[2][2].im) * 0.57735026918962576451;   // 1/sqrt(3)
}

// A block covers 64 sites and its wave w computes direction w (a wave-uniform
// branch), so each thread holds one direction's operands; the four waves read
// the same X(x), Y(x) (cache hits after the first; staging them in LDS once per
// block measured 3 % slower).  Projecting every spinor as it arrives and adding
// each outer product to Q at once would fit 168 registers (three waves per SIMD),
// but at that budget the compiler waits for each spinor's loads before issuing
// the next one's.  Compiled for at most two waves per SIMD (about 205 registers)
// it issues them together: 39 -> 35 us at 16^3 x 32, 191 -> 185 us at 24^3 x 48
// and 612 -> 559 us at 32^3 x 64, bitwise the same output.  Holding all four
// directions per thread needed 260 registers, one wave per SIMD, and ran 14 %
// slower; putting the two terms of Q on separate waves (eight per block, four
// waves per SIMD with 36 registers spilled) ran 45 % slower.
template <int R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void force_dir_kernel(const ForceK a) {
    // the block's 64 output records (32 doubles each, +1 against bank conflicts) and their sites
    __shared__ double otile[64][33];
    __shared__ int64_t srec[64];
    const int lane = threadIdx.x & 63;
    const int mu = threadIdx.x >> 6;
    int par, h;
    if (force_block_site(a, blockIdx.x, lane, par, h)) {
        const int lxh = a.lxh, lx = a.L[0], ly = a.L[1], lz = a.L[2], lt = a.L[3];
        const int xh = h % lxh;
        int rest = h / lxh;
        const int y = rest % ly;
        rest /= ly;
        const int z = rest % lz;
        const int t = rest / lz;
        const int bit = (par + y + z + t) & 1;
        const int x = 2 * xh + bit;

        double g[8];
        if (mu == 0) {
            const int xf = x + 1 == lx ? 0 : x + 1;
            force_dir<R, 0>(a, par, h, (h - xh) + (xf >> 1), x == lx - 1, g);
        } else if (mu == 1) {
            const int nf = y == ly - 1 ? h - (ly - 1) * lxh : h + lxh;
            force_dir<R, 1>(a, par, h, nf, y == ly - 1, g);
        } else if (mu == 2) {
            const int st = lxh * ly;
            const int nf = z == lz - 1 ? h - (lz - 1) * st : h + st;
            force_dir<R, 2>(a, par, h, nf, z == lz - 1, g);
        } else {
            const int st = lxh * ly * lz;
            const int nf = t == lt - 1 ? h - (lt - 1) * st : h + st;
            force_dir<R, 3>(a, par, h, nf, t == lt - 1, g);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) otile[lane][mu * 8 + i] = a.scale * g[i];
        if (mu == 0) srec[lane] = 2 * (int64_t)h + bit;
    } else if (mu == 0) {
        srec[lane] = -1;
    }
    __syncthreads();
    // each record is 256 contiguous bytes of the canonical [V][4][8] output: a wave
    // writes four whole records in 16-byte units instead of 64 scattered 8-byte words.
    // Nontemporal: the launch never reads them back, and kept out of the L2 they leave
    // it to the X, Y it still reads (212 -> 193 us at 24^3 x 48, 627 -> 616 us at 32^3 x 64)
    for (int u = threadIdx.x; u < 64 * 16; u += kBlock) {
        const int rec = u >> 4, k = u & 15;
        const int64_t sr = srec[rec];
        if (sr < 0) continue;
        double2* o = reinterpret_cast<double2*>(a.out + sr * 32) + k;
        double2 v = make_double2(otile[rec][2 * k], otile[rec][2 * k + 1]);
        if (a.accumulate) {
            const double2 w = *o;
            v.x = w.x + v.x;
            v.y = w.y + v.y;
        }
        st_stream(o, v);
    }
}

}  // namespace

hipError_t launch_force(const Geom& g, const void* gauge, int recon, const void* const X[2], const void* const Y[2],
                        double* out, const Cplx bc[4], double kappa, double scale, int accumulate, hipStream_t s) {
    ForceK k;
    k.gauge = static_cast<const char*>(gauge);
    for (int p = 0; p < 2; ++p) {
        k.X[p] = static_cast<const char*>(X[p]);
        k.Y[p] = static_cast<const char*>(Y[p]);
    }
    k.out = out;
    k.stride = g.stride;
    k.gstride = g.gstride;
    for (int i = 0; i < 4; ++i) {
        k.L[i] = g.L[i];
        k.bc[i] = {bc[i].re, bc[i].im};
    }
    k.lxh = g.lxh;
    k.vh = (int)g.vh;
    k.kappa = kappa;
    k.scale = scale;
    k.accumulate = accumulate;
    k.lt = g.L[3];
    k.slice = (int)(g.vh / g.L[3]);
    k.q = (k.slice + kNumXcd - 1) / kNumXcd;
    k.tq = (k.q + 63) / 64;
    const dim3 grid(2 * kNumXcd * k.lt * k.tq);
    switch (recon) {
        case TMQCD_RECON18: hipLaunchKernelGGL((force_dir_kernel<TMQCD_RECON18>), grid, dim3(kBlock), 0, s, k); break;
        case TMQCD_RECON12: hipLaunchKernelGGL((force_dir_kernel<TMQCD_RECON12>), grid, dim3(kBlock), 0, s, k); break;
        case TMQCD_RECON10: hipLaunchKernelGGL((force_dir_kernel<TMQCD_RECON10>), grid, dim3(kBlock), 0, s, k); break;
        case TMQCD_RECON8: hipLaunchKernelGGL((force_dir_kernel<TMQCD_RECON8>), grid, dim3(kBlock), 0, s, k); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tmqcd
