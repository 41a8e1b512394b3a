"""FP64 oracle for the paper's tree-level Symanzik gauge action and its force.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.

* Action (the paper's gauge-sector equation, in the normalisation
  (beta/3)(3 - Re Tr) per loop used throughout):
      S = (beta/3) sum_x [ c0 sum_{mu<nu} (3 - Re Tr P_mu_nu(x))
                         + c1 sum_{mu != nu} (3 - Re Tr R_mu_nu(x)) ],   c0 = 1 - 8 c1,
  with R_mu_nu(x) the 2x1 rectangle two links long in mu and one in nu,
      R_mu_nu(x) = U_mu(x) U_mu(x+mu) U_nu(x+2mu) U_mu(x+mu+nu)^+ U_mu(x+nu)^+ U_nu(x)^+.
  Each geometric rectangle is counted once: it has one long direction mu, one
  short direction nu and one corner x with both edges leaving it forwards.
  The paper prints c1 = 1/12; tree-level improvement needs c1 = -1/12 (then the
  constant-field expansion has no O(a^2) term), and that is the reading taken.
* Force, as for the plaquette action: G^a = (beta/3) Im Tr[T^a U_mu(x) V_mu(x)]
  with V_mu(x) = c0 (sum of the 6 plaquette staples) + c1 (sum of the 18
  rectangle staples).  A staple is the product of the other links of a closed
  loop through U_mu(x), walked from x+mu back to x, so that the loop's trace is
  Tr[U_mu(x) V]; every loop through the link is walked in the sense in which it
  runs forwards over the link (Re Tr is the same for both senses).
Loops are built here by walking explicit lists of steps (+d forwards over
U_d(y), -d backwards over U_d(y - d)^+); nothing is shared with force.py.
"""
from __future__ import annotations

import numpy as np

from .dirac import AXIS, shape4
from .force import T_GEN

__all__ = ["walk", "loop_trace_sum", "plaquette_sum", "rectangle_sum", "action", "staple_sum", "force",
           "PLAQUETTE_STAPLE_PATHS", "RECTANGLE_STAPLE_PATHS"]


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def _at(field, offset):
    """field(x + offset) for every x (periodic); field has the four lattice axes first."""
    out = field
    for d in range(4):
        if offset[d]:
            out = np.roll(out, -offset[d], axis=AXIS[d])
    return out


def walk(u, start, steps):
    """Product of the links along the path from x + start taking `steps` (signed 1-based directions:
    +(d+1) forwards along d, -(d+1) backwards), for every x.  u: (lattice..., 4, 3, 3)."""
    pos = list(start)
    prod = None
    for st in steps:
        d = abs(st) - 1
        if st > 0:
            m = _at(u[..., d, :, :], pos)
            pos[d] += 1
        else:
            pos[d] -= 1
            m = _dag(_at(u[..., d, :, :], pos))
        prod = m if prod is None else prod @ m
    return prod


def _closed(steps):
    tot = [0, 0, 0, 0]
    for st in steps:
        tot[abs(st) - 1] += 1 if st > 0 else -1
    return tot == [0, 0, 0, 0]


def loop_trace_sum(U, dims, steps) -> float:
    """sum_x Re Tr of the closed loop `steps` from x."""
    assert _closed(steps)
    u = U.reshape(shape4(dims) + (4, 3, 3))
    return float(np.trace(walk(u, (0, 0, 0, 0), steps), axis1=-2, axis2=-1).real.sum())


def plaquette_sum(U, dims) -> float:
    """sum_{x, mu<nu} Re Tr P_mu_nu(x)."""
    return sum(loop_trace_sum(U, dims, [m + 1, n + 1, -(m + 1), -(n + 1)])
               for m in range(4) for n in range(m + 1, 4))


def rectangle_sum(U, dims) -> float:
    """sum_{x, mu != nu} Re Tr R_mu_nu(x) (two links along mu, one along nu)."""
    return sum(loop_trace_sum(U, dims, [m + 1, m + 1, n + 1, -(m + 1), -(m + 1), -(n + 1)])
               for m in range(4) for n in range(4) if n != m)


def action(U, dims, beta, c1) -> float:
    v = int(np.prod(dims))
    c0 = 1.0 - 8.0 * c1
    return float(beta / 3.0 * (c0 * (3.0 * 6 * v - plaquette_sum(U, dims))
                               + c1 * (3.0 * 12 * v - rectangle_sum(U, dims))))


def _staple_paths(mu):
    """The rest of every plaquette and every rectangle loop through U_mu(x), walked forwards over the link,
    as step lists from x + mu back to x."""
    m = mu + 1
    plaq, rect = [], []
    for nu in range(4):
        if nu == mu:
            continue
        for s in (nu + 1, -(nu + 1)):
            plaq.append([s, -m, -s])
            rect.append([m, s, -m, -m, -s])     # long along mu, the link first
            rect.append([s, -m, -m, -s, m])     # long along mu, the link second
            rect.append([s, s, -m, -s, -s])     # long along nu
    return plaq, rect


PLAQUETTE_STAPLE_PATHS = {mu: _staple_paths(mu)[0] for mu in range(4)}
RECTANGLE_STAPLE_PATHS = {mu: _staple_paths(mu)[1] for mu in range(4)}


def staple_sum(U, dims, c1) -> np.ndarray:
    """V_mu(x) = c0 (6 plaquette staples) + c1 (18 rectangle staples), shape (V, 4, 3, 3)."""
    u = U.reshape(shape4(dims) + (4, 3, 3))
    c0 = 1.0 - 8.0 * c1
    v = np.zeros_like(u)
    for mu in range(4):
        start = [0, 0, 0, 0]
        start[mu] = 1
        for p in PLAQUETTE_STAPLE_PATHS[mu]:
            assert _closed([mu + 1] + p)
            v[..., mu, :, :] += c0 * walk(u, start, p)
        if c1 != 0.0:
            for p in RECTANGLE_STAPLE_PATHS[mu]:
                assert _closed([mu + 1] + p)
                v[..., mu, :, :] += c1 * walk(u, start, p)
    return v.reshape(-1, 4, 3, 3)


def force(U, dims, beta, c1) -> np.ndarray:
    """dS/dw^a of the tree-level Symanzik action, shape (V, 4, 8)."""
    uv = U @ staple_sum(U, dims, c1)
    return beta / 3.0 * np.einsum("aij,...ji->...a", T_GEN, uv).imag
