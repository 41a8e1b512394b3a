"""FP64 oracle for BiCGStab, the paper's other Krylov solver (§2.1: the inversion D phi = psi
is done with CG or BiCGStab).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.

BiCGStab (van der Vorst, SIAM J. Sci. Stat. Comput. 13 (1992) 631) solves a
general non-singular system A x = b, so it applies to M (or the even-odd Schur
complement Mhat) directly instead of the normal operator.  With the shadow
residual rt = r_0 and rho_0 = alpha_0 = omega_0 = 1, v_0 = p_0 = 0, for i = 1, 2, ...:
    rho_i   = (rt, r_{i-1})
    beta    = (rho_i / rho_{i-1}) (alpha / omega_{i-1})
    p_i     = r_{i-1} + beta (p_{i-1} - omega_{i-1} v_{i-1})
    v_i     = A p_i
    alpha   = rho_i / (rt, v_i)
    s       = r_{i-1} - alpha v_i
    t       = A s
    omega_i = (t, s) / (t, t)
    x_i     = x_{i-1} + alpha p_i + omega_i s
    r_i     = s - omega_i t
(x, y) = x^dag y.  It stops when ||r_i|| <= tol ||b|| (the recursive residual;
the caller recomputes the true one).
"""
from __future__ import annotations

import numpy as np

__all__ = ["bicgstab"]


def bicgstab(apply_A, b, tol: float = 1e-10, maxiter: int = 100000, x0=None):
    """Returns (x, iterations, converged)."""
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128, copy=True)
    r = b - apply_A(x) if x0 is not None else b.copy()
    rt = r.copy()
    bb = np.vdot(b, b).real
    if bb == 0.0:
        return np.zeros_like(b), 0, True
    rho_prev = alpha = omega = 1.0 + 0.0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    k = 0
    while np.vdot(r, r).real > tol * tol * bb:
        if k >= maxiter:
            return x, k, False
        rho = np.vdot(rt, r)
        beta = (rho / rho_prev) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply_A(p)
        alpha = rho / np.vdot(rt, v)
        s = r - alpha * v
        t = apply_A(s)
        tt = np.vdot(t, t).real
        omega = np.vdot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_prev = rho
        k += 1
    return x, k, True
