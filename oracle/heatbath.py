"""FP64 oracle for the pure-gauge heatbath and overrelaxation updates (the paper's heatbath section).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.

Action: the Wilson plaquette action S = (beta/3) sum_{x, mu<nu} (3 - Re Tr P), so
a link U = U_mu(x) with staple sum V (force.staple_sum: the plaquettes through
the link sum to Re Tr[U V]) has the local weight exp((beta/3) Re Tr[U V]).

One SU(3) update runs over the SU(2) subgroups (rows/columns (0,1), (0,2),
(1,2)), as the paper's sketch does (project, update, extend, multiply):
  * W = U V; its 2x2 block w on the subgroup's rows and columns; the quaternion
    part of w, q = a0 + i a.sigma with a0 = Re(w00 + w11)/2, a1 = Im(w01 + w10)/2,
    a2 = Re(w01 - w10)/2, a3 = Im(w00 - w11)/2, is q = k s with k = |a| and s in
    SU(2) (the rest of w drops out of Re Tr[r w] for r in SU(2));
  * heatbath: draw x in SU(2) with weight exp(alpha x0), alpha = (2/3) beta k,
    and set r = x s^+, so that r has weight exp((beta/3) Re Tr[r w]);
  * overrelaxation: r = (s^+)^2, which leaves Re Tr[r w] = Re Tr[w] unchanged;
  * extend r to the subgroup's rows and columns of the identity R and set
    U <- R U (the sketch's multiplication, taken from the left so that the new
    W is R W).
x0 is drawn with density sqrt(1 - x0^2) exp(alpha x0) on [-1, 1] (Haar measure
on SU(2) times the weight): for alpha < 2 by inverting the exponential
(x0 = -1 + log1p(u expm1(2 alpha)) / alpha, accepted with probability
sqrt(1 - x0^2); Creutz 1980), else by Kennedy and Pendleton's method
(lambda^2 = -(log r1 + cos^2(2 pi r2) log r3) / (2 alpha), accepted when
r4^2 <= 1 - lambda^2, x0 = 1 - 2 lambda^2; Kennedy and Pendleton 1985).  The
direction of (x1, x2, x3) is uniform on the sphere: cos(theta) = 2 u1 - 1,
phi = 2 pi u2.  alpha = 0 gives x0 = 2u - 1 accepted with sqrt(1 - x0^2).
1 - x^2 is evaluated as (1 - x)(1 + x), which stays accurate to a few units
in the last place near x = +-1, where the square root magnifies the error of
1 - x x by 1/sqrt(1 - x^2).

A sweep updates every link, direction by direction and parity by parity: the
staples of U_mu(x) hold no other U_mu(y) of the parity of x, so those links are
independent given the rest.

Random numbers come from the counter-based generator Philox4x32-10 (Salmon,
Moraes, Dror and Shaw, SC'11), written here from its definition: 10 rounds of
  (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
M0 = 0xD2511F53, M1 = 0xCD9E8D57, the key (k0, k1) raised by (0x9E3779B9,
0xBB67AE85) after every round.  Key = (seed mod 2^32, seed div 2^32); counter
= (4 s + mu, sweep, subgroup * 2^16 + trial, 0) with s the canonical site
index; the direction uses trial 0xFFFF.  A 32-bit word w becomes the uniform
(w + 1/2) 2^-32 in (0, 1).  A trial of the alpha < 2 method uses words 0 and 1
(u, then the acceptance uniform), one of Kennedy-Pendleton words 0..3 (r1..r4).
"""
from __future__ import annotations

import numpy as np

from .dirac import coords
from .force import staple_sum

__all__ = ["philox4x32", "uniform", "sample_x0", "su2_project", "update_su3", "heatbath_sweep", "overrelax_sweep",
           "SUBGROUPS", "ALPHA_SWITCH", "DIR_TRIAL"]

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF
SUBGROUPS = ((0, 1), (0, 2), (1, 2))
ALPHA_SWITCH = 2.0
DIR_TRIAL = 0xFFFF


def philox4x32(c0, c1, c2, c3, k0, k1, rounds: int = 10):
    """Philox4x32 on arrays of uint64 holding 32-bit values; returns four uint64 arrays."""
    c = [np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for i in range(rounds):
        p0 = np.uint64(M0) * c[0]           # 32 x 32 -> 64 bits, exact in uint64
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        if i < rounds - 1:
            k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
            k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return c


def uniform(w):
    """(w + 1/2) 2^-32 for 32-bit words w: in (0, 1), exact in FP64."""
    return (w.astype(np.float64) + 0.5) * 2.0 ** -32


def _words(seed, link, sweep, sub, trial):
    k0, k1 = np.uint64(seed & MASK), np.uint64((seed >> 32) & MASK)
    c2 = np.uint64(sub << 16) + np.asarray(trial, dtype=np.uint64)
    return philox4x32(link, np.uint64(sweep), c2, np.uint64(0), k0, k1)


def sample_x0(alpha, seed, link, sweep, sub, max_trials: int = 0xFFFE, flips=None, watch=None):
    """x0 with density sqrt(1 - x0^2) exp(alpha x0) on [-1, 1], one per link (arrays alpha, link).

    Decisions of the sampler are (link, sub, -1) for the choice of method (alpha < 2) and
    (link, sub, t) for the acceptance of trial t.  Two test hooks, unused by default:
    `flips`, a set of decisions taken the other way; `watch`, a dict {link: list} to which
    the margin of every decision made for that link is appended as ((link, sub, t), margin),
    the margin being positive for "yes" and its size the distance to the other outcome
    (alpha - 2 for the method; sqrt(1 - x0^2) - u, or 1 - lambda^2 - r4^2, for a trial)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    link_ids = np.atleast_1d(np.asarray(link, dtype=np.uint64)).astype(np.int64)
    x0 = np.zeros_like(alpha)
    todo = np.ones(alpha.shape, dtype=bool)
    small = alpha < ALPHA_SWITCH

    def flipped(i, t):
        return flips is not None and (int(link_ids[i]), sub, t) in flips

    watched = [] if watch is None else [i for i, l in enumerate(link_ids) if int(l) in watch]
    for i in watched:
        watch[int(link_ids[i])].append(((int(link_ids[i]), sub, -1), float(ALPHA_SWITCH - alpha[i])))
    if flips:
        for i in range(len(link_ids)):
            if flipped(i, -1):
                small[i] = not small[i]
    for trial in range(max_trials):
        if not todo.any():
            break
        w = _words(seed, link, sweep, sub, trial)
        u = [uniform(v) for v in w]
        with np.errstate(divide="ignore", invalid="ignore"):
            # alpha < 2: invert the exponential, accept with sqrt(1 - x0^2)
            xc = np.where(alpha > 0, -1.0 + np.log1p(u[0] * np.expm1(2.0 * alpha)) / np.where(alpha > 0, alpha, 1.0),
                          2.0 * u[0] - 1.0)
            marg_c = np.sqrt(np.maximum(0.0, (1.0 - xc) * (1.0 + xc))) - u[1]
            acc_c = marg_c >= 0
            # Kennedy-Pendleton
            lam2 = -(np.log(u[0]) + np.cos(2.0 * np.pi * u[1]) ** 2 * np.log(u[2])) / (2.0 * alpha)
            marg_k = (1.0 - lam2) - u[3] * u[3]
            acc_k = marg_k >= 0
            xk = 1.0 - 2.0 * lam2
        acc = np.where(small, acc_c, acc_k)
        for i in watched:
            if todo[i]:
                m = marg_c[i] if small[i] else marg_k[i]
                watch[int(link_ids[i])].append(((int(link_ids[i]), sub, trial), float(m)))
        if flips:
            for i in np.nonzero(todo)[0]:
                if flipped(i, trial):
                    acc[i] = not acc[i]
        acc &= todo
        x0 = np.where(acc, np.where(small, xc, xk), x0)
        todo &= ~acc
    if todo.any():
        raise RuntimeError("x0 sampler exceeded its trial cap")
    return x0


def su2_project(w):
    """Quaternion part (a0, a1, a2, a3) of 2x2 blocks w[..., 2, 2]."""
    a0 = 0.5 * (w[..., 0, 0] + w[..., 1, 1]).real
    a1 = 0.5 * (w[..., 0, 1] + w[..., 1, 0]).imag
    a2 = 0.5 * (w[..., 0, 1] - w[..., 1, 0]).real
    a3 = 0.5 * (w[..., 0, 0] - w[..., 1, 1]).imag
    return a0, a1, a2, a3


def _su2(a0, a1, a2, a3):
    """The 2x2 matrix a0 + i (a1 sigma1 + a2 sigma2 + a3 sigma3)."""
    m = np.empty(np.shape(a0) + (2, 2), dtype=np.complex128)
    m[..., 0, 0] = a0 + 1j * a3
    m[..., 0, 1] = a2 + 1j * a1
    m[..., 1, 0] = -a2 + 1j * a1
    m[..., 1, 1] = a0 - 1j * a3
    return m


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def update_su3(u, V, beta, seed: int, link, sweep: int, heatbath: bool, flips=None, watch=None):
    """Update links u[n, 3, 3] with staple sums V[n, 3, 3] over the three subgroups; link[n] are their
    generator ids (4 s + mu).  Returns the new links.  flips, watch: the test hooks of sample_x0."""
    u = u.copy()
    for sub, (a, b) in enumerate(SUBGROUPS):
        W = u @ V
        blk = W[:, [a, b]][:, :, [a, b]]
        a0, a1, a2, a3 = su2_project(blk)
        k = np.sqrt(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3)
        nz = k > 0
        ks = np.where(nz, k, 1.0)
        s = _su2(np.where(nz, a0 / ks, 1.0), np.where(nz, a1 / ks, 0.0), np.where(nz, a2 / ks, 0.0),
                 np.where(nz, a3 / ks, 0.0))
        if heatbath:
            alpha = (2.0 / 3.0) * beta * k
            x0 = sample_x0(alpha, seed, link, sweep, sub, flips=flips, watch=watch)
            wd = _words(seed, link, sweep, sub, DIR_TRIAL)
            cth = 2.0 * uniform(wd[0]) - 1.0
            phi = 2.0 * np.pi * uniform(wd[1])
            rad = np.sqrt(np.maximum(0.0, (1.0 - x0) * (1.0 + x0)))
            sth = np.sqrt(np.maximum(0.0, (1.0 - cth) * (1.0 + cth)))
            x = _su2(x0, rad * sth * np.cos(phi), rad * sth * np.sin(phi), rad * cth)
            r = x @ _dag(s)
        else:
            sd = _dag(s)
            r = np.where(nz[:, None, None], sd @ sd, np.eye(2, dtype=np.complex128))
        ua, ub = u[:, a, :].copy(), u[:, b, :].copy()
        u[:, a, :] = r[:, 0, 0, None] * ua + r[:, 0, 1, None] * ub
        u[:, b, :] = r[:, 1, 0, None] * ua + r[:, 1, 1, None] * ub
    return u


def _update_links(U, dims, beta, seed, sweep, heatbath: bool, flips=None, watch=None):
    """One sweep over directions and parities; returns the new links (V, 4, 3, 3)."""
    U = U.copy()
    parity = coords(dims).sum(axis=1) % 2
    for mu in range(4):
        for par in (0, 1):
            sites = np.nonzero(parity == par)[0]
            V = staple_sum(U, dims)[sites, mu]
            link = (4 * sites + mu).astype(np.uint64)
            U[sites, mu] = update_su3(U[sites, mu], V, beta, seed, link, sweep, heatbath, flips, watch)
    return U


def heatbath_sweep(U, dims, beta, seed: int, sweep: int, flips=None, watch=None):
    """One heatbath sweep with the generator streams of (seed, sweep).  flips, watch: the test
    hooks of sample_x0 (decisions taken the other way; margins of a link's decisions)."""
    return _update_links(U, dims, beta, seed, sweep, True, flips, watch)


def overrelax_sweep(U, dims):
    """One overrelaxation sweep (no random numbers; independent of beta)."""
    return _update_links(U, dims, 0.0, 0, 0, False)
