"""FP64 oracle for the leapfrog hybrid Monte-Carlo of the paper's ensemble-generation section.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.

* H = 1/2 sum (p^a)^2 + S_g + S_f with momenta P_mu(x) = p^a T^a (8 reals per link).
* Equations of motion dU/dt = i P U and dp^a/dt = -G^a = F^a (the paper's
  P-dot = -dS/dU, U-dot = P in the left-multiplied parametrisation).
* Leapfrog over n steps of dt: half momentum step, then n times (full link step,
  momentum step), the last momentum step being a half step.
* Pseudofermion refresh phi = M^dag eta with eta complex Gaussian, so that
  phi^dag (M^dag M)^{-1} phi = eta^dag eta is Gaussian-distributed as detailed
  balance requires.
* Metropolis: accept with probability min(1, exp(-(H' - H))); the paper prints
  the exponent without its minus sign.
* The paper's production integrator (its HMC section): the second-order
  minimal-norm (2MN, Omelyan) scheme on two timescales, the fermion force on
  the outer scale and the gauge force on the inner one (Sexton-Weingarten
  nesting).  One outer step of dt, with lam = 0.1931833275037836:
      p -= lam dt G_f;  inner(dt/2);  p -= (1 - 2 lam) dt G_f;  inner(dt/2);  p -= lam dt G_f
  and inner(tau) = n_inner steps of h = tau/n_inner of the same scheme with the
  gauge force and the link updates U <- exp(i (h/2) p^a T^a) U in place of inner.
  Without a gauge force inner(tau) is the link update over tau.
* Even-odd HMC: the pseudofermion lives on even sites, phi_e = Mhat^dag eta_e,
  and the action is S_f^eo (see force.py).  Its gauge action is the tree-level
  Symanzik one of symanzik.py with coefficient c1 (c1 = 0: the Wilson action).
Random numbers (momenta, eta, the Metropolis uniform) are inputs.
"""
from __future__ import annotations

import numpy as np

from .dirac import apply_M, apply_Mdag, apply_MdagM, apply_Mhatdag, apply_MhatdagMhat, cg
from . import symanzik
from .force import T_GEN, fermion_force, fermion_force_eo, gauge_action, gauge_force

__all__ = ["su3_exp", "hamiltonian", "total_gradient", "leapfrog", "trajectory", "LAMBDA_2MN", "omelyan",
           "hamiltonian_eo", "trajectory_eo"]

LAMBDA_2MN = 0.1931833275037836


def su3_exp(p, dt) -> np.ndarray:
    """exp(i dt p^a T^a) for p of shape (..., 8), by diagonalising the hermitian generator."""
    h = np.einsum("...a,aij->...ij", p, T_GEN)
    w, v = np.linalg.eigh(h)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * dt * w), v.conj())


class _Action:
    def __init__(self, dims, kappa, mu, bc, beta, tol):
        self.dims, self.kappa, self.mu, self.bc, self.beta, self.tol = dims, kappa, mu, bc, beta, tol

    def solve(self, U, phi):
        a = lambda v: apply_MdagM(U, v, self.dims, self.kappa, self.mu, self.bc)
        x, _ = cg(a, phi, self.tol)
        return x

    def s_fermion(self, U, phi):
        return float(np.vdot(phi, self.solve(U, phi)).real)

    def gradient(self, U, phi):
        x = self.solve(U, phi)
        y = apply_M(U, x, self.dims, self.kappa, self.mu, self.bc)
        g = fermion_force(U, x, y, self.dims, self.kappa, self.bc)
        if self.beta != 0:
            g = g + gauge_force(U, self.dims, self.beta)
        return g


def hamiltonian(U, p, phi, dims, kappa, mu, bc, beta, tol=1e-14) -> float:
    act = _Action(dims, kappa, mu, bc, beta, tol)
    h = 0.5 * float(np.sum(p * p)) + act.s_fermion(U, phi)
    if beta != 0:
        h += gauge_action(U, dims, beta)
    return h


def total_gradient(U, phi, dims, kappa, mu, bc, beta, tol=1e-14) -> np.ndarray:
    return _Action(dims, kappa, mu, bc, beta, tol).gradient(U, phi)


def leapfrog(U, p, phi, dims, kappa, mu, bc, beta, n_steps, dt, tol=1e-14):
    """Integrate (U, p) over n_steps * dt; returns new copies."""
    act = _Action(dims, kappa, mu, bc, beta, tol)
    u = U.copy()
    q = p - 0.5 * dt * act.gradient(u, phi)
    for i in range(n_steps):
        u = su3_exp(q, dt) @ u
        step = dt if i < n_steps - 1 else 0.5 * dt
        q = q - step * act.gradient(u, phi)
    return u, q


def trajectory(U, p, eta, uniform, dims, kappa, mu, bc, beta, n_steps, dt, tol=1e-14):
    """One HMC trajectory.  Returns dict(U, accepted, dH, H0, H1, phi)."""
    phi = apply_Mdag(U, eta, dims, kappa, mu, bc)
    h0 = hamiltonian(U, p, phi, dims, kappa, mu, bc, beta, tol)
    u1, p1 = leapfrog(U, p, phi, dims, kappa, mu, bc, beta, n_steps, dt, tol)
    h1 = hamiltonian(u1, p1, phi, dims, kappa, mu, bc, beta, tol)
    dh = h1 - h0
    accepted = bool(uniform < np.exp(-dh))
    return {"U": u1 if accepted else U, "accepted": accepted, "dH": dh, "H0": h0, "H1": h1,
            "phi": phi, "U_proposed": u1, "p_proposed": p1}


class _ActionEO:
    """The even-odd pseudofermion action and, separately, the tree-level Symanzik gauge action."""

    def __init__(self, dims, kappa, mu, bc, beta, tol, c1=0.0):
        self.dims, self.kappa, self.mu, self.bc, self.beta, self.tol = dims, kappa, mu, bc, beta, tol
        self.c1 = c1

    def solve(self, U, phi_e):
        a = lambda v: apply_MhatdagMhat(U, v, self.dims, self.kappa, self.mu, self.bc)
        x, _ = cg(a, phi_e, self.tol)
        return x

    def s_fermion(self, U, phi_e):
        return float(np.vdot(phi_e, self.solve(U, phi_e)).real)

    def fermion_gradient(self, U, phi_e):
        return fermion_force_eo(U, self.solve(U, phi_e), self.dims, self.kappa, self.mu, self.bc)

    def gauge_gradient(self, U):
        return symanzik.force(U, self.dims, self.beta, self.c1)

    def s_gauge(self, U):
        return symanzik.action(U, self.dims, self.beta, self.c1)


def omelyan(U, p, grad_outer, grad_inner, n_outer, dt, n_inner=1, lam=LAMBDA_2MN):
    """Two-level 2MN integration of (U, p) over n_outer * dt; returns new copies.

    grad_outer(U) is the gradient integrated on the outer scale, grad_inner(U)
    (or None) the one integrated on the inner scale.
    """
    def inner(u, q, tau):
        if grad_inner is None:
            return su3_exp(q, tau) @ u, q
        h = tau / n_inner
        for _ in range(n_inner):
            q = q - lam * h * grad_inner(u)
            u = su3_exp(q, 0.5 * h) @ u
            q = q - (1.0 - 2.0 * lam) * h * grad_inner(u)
            u = su3_exp(q, 0.5 * h) @ u
            q = q - lam * h * grad_inner(u)
        return u, q

    u, q = U.copy(), p.copy()
    for _ in range(n_outer):
        q = q - lam * dt * grad_outer(u)
        u, q = inner(u, q, 0.5 * dt)
        q = q - (1.0 - 2.0 * lam) * dt * grad_outer(u)
        u, q = inner(u, q, 0.5 * dt)
        q = q - lam * dt * grad_outer(u)
    return u, q


def hamiltonian_eo(U, p, phi_e, dims, kappa, mu, bc, beta, tol=1e-14, c1=0.0) -> float:
    act = _ActionEO(dims, kappa, mu, bc, beta, tol, c1)
    h = 0.5 * float(np.sum(p * p)) + act.s_fermion(U, phi_e)
    if beta != 0:
        h += act.s_gauge(U)
    return h


def trajectory_eo(U, p, eta_e, uniform, dims, kappa, mu, bc, beta, n_outer, dt, n_inner=1, tol=1e-14, c1=0.0):
    """One even-odd HMC trajectory with the two-level 2MN integrator (fermion force outer, gauge force of
    the tree-level Symanzik action with coefficient c1 inner).

    Returns dict(U, accepted, dH, H0, H1, phi_e, U_proposed, p_proposed)."""
    act = _ActionEO(dims, kappa, mu, bc, beta, tol, c1)
    phi_e = apply_Mhatdag(U, eta_e, dims, kappa, mu, bc)
    h0 = hamiltonian_eo(U, p, phi_e, dims, kappa, mu, bc, beta, tol, c1)
    grad_inner = act.gauge_gradient if beta != 0 else None
    u1, p1 = omelyan(U, p, lambda u: act.fermion_gradient(u, phi_e), grad_inner, n_outer, dt, n_inner)
    h1 = hamiltonian_eo(u1, p1, phi_e, dims, kappa, mu, bc, beta, tol, c1)
    dh = h1 - h0
    accepted = bool(uniform < np.exp(-dh))
    return {"U": u1 if accepted else U, "accepted": accepted, "dH": dh, "H0": h0, "H1": h1,
            "phi_e": phi_e, "U_proposed": u1, "p_proposed": p1}
