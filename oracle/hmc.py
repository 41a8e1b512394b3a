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
Random numbers (momenta, eta, the Metropolis uniform) are inputs.
"""
from __future__ import annotations

import numpy as np

from .dirac import apply_M, apply_Mdag, apply_MdagM, cg
from .force import T_GEN, fermion_force, gauge_action, gauge_force

__all__ = ["su3_exp", "hamiltonian", "total_gradient", "leapfrog", "trajectory"]


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
