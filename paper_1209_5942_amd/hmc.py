"""Leapfrog hybrid Monte-Carlo and the differentiable pseudofermion action on the HIP library.

Paper, ensemble-generation section: H = 1/2 P^2 + S_g + S_f with momenta P
conjugate to U, evolved with a symplectic integrator and followed by a
Metropolis step.  Here:

* S_f = phi^+ (M^+ M)^{-1} phi on the full lattice, phi = M^+ eta refreshed
  from a Gaussian eta (random numbers are inputs);
* S_g = (beta/3) sum_{x,mu<nu} (3 - Re Tr P_mu_nu) (the tree-level Symanzik
  action at c1 = 0);
* leapfrog: half momentum step, n times (link step, momentum step), the last
  momentum step a half step; U <- exp(i dt p^a T^a) U; p <- p - dt G;
* Metropolis: accept with probability min(1, exp(-(H' - H))).

Every step runs in libtmqcd kernels (CG, force, gauge force, link update,
reductions); torch provides device buffers and the copies that keep the
rejected configuration.  :class:`FermionAction` exposes S_f to autograd: its
backward pass is the fermion-force kernel.
"""
from __future__ import annotations

import math

import torch

from . import tmqcd as T


class FermionAction(torch.autograd.Function):
    """S_f(omega) = phi^+ (M^+ M)^{-1} phi at links exp(i omega^a T^a) U.

    forward(omega, ctx_obj) with omega a float64 device tensor (V, 4, 8) and
    ctx_obj a :class:`HMC`; returns a 0-dim float64 tensor.  The backward pass
    returns the fermion force G evaluated at the links exp(i omega.T) U: the
    derivative of S_f along left translations there, equal to dS_f/domega at
    omega = 0 (where HMC evaluates it).
    """

    @staticmethod
    def forward(ctx, omega, h: "HMC"):
        U = h.U
        if bool(torch.any(omega != 0)):
            U = h.U.clone()
            T.update_links(h.prob, U, omega, 1.0)
        X = h.solve(h.phi, U)
        s = T.dot(h.prob, h.phi, X, T.FULL, ws=h.ws_aux)
        ctx.h, ctx.U, ctx.X = h, U, X
        return s[0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        h = ctx.h
        Y = T.dslash(h.prob, ctx.U, ctx.X, T.M, ws=h.ws_dslash)
        G = T.force(h.prob, ctx.U, ctx.X, Y, scale=float(grad_out))
        return G, None


class HMC:
    """Two-flavour twisted-mass HMC state on one GPU: packed FP64 links and solver buffers.

    inner_prec: storage precision of the hops inside every solve (T.F64: plain
    FP64 CG; T.F32 or T.F16: defect correction with reliable updates to the
    same FP64 tolerance on the true residual).  A low-precision copy of the
    links is packed from the FP64 links whenever they change.

    guess: start every solve with the same right-hand side phi from the last
    solution instead of zero (the links moved by one step since); the result
    still meets the tolerance on the true residual, so only the iteration
    count changes (and, at the level of the tolerance, the reversibility).
    """

    def __init__(self, prob: T.Problem, U_canon, beta: float, tol: float = 1e-12, max_iter: int = 20000,
                 md_tol: float | None = None, inner_prec: int = T.F64, guess: bool = False):
        self.prob = prob
        self.beta = float(beta)
        self.tol = tol                      # solves that enter H (acceptance)
        self.md_tol = md_tol or tol         # solves that enter the force
        self.max_iter = max_iter
        self.inner = inner_prec
        self.guess = guess
        self._have_x = False      # self.X holds a solution for the current phi
        self.U = T.pack_gauge(prob, U_canon, T.F64, T.RECON18)
        self.U_low = None
        self.refresh_low()
        dev = self.U.device
        fb = T.spinor_bytes(prob, T.F64, T.FULL)
        self.ws_cg = T.workspace(prob, T.MDAGM, 1 | (1 << inner_prec))
        self.ws_dslash = T.workspace(prob, T.MDAGM, 1)
        self.ws_aux = T.aux_workspace(prob)
        self.X = torch.empty(fb, dtype=torch.uint8, device=dev)
        self.Y = torch.empty(fb, dtype=torch.uint8, device=dev)
        self.phi = torch.empty(fb, dtype=torch.uint8, device=dev)
        self.solves = 0
        self.cg_iters = 0

    # --------------------------------------------------------------- pieces ---
    def set_pseudofermion(self, eta_canon):
        """phi = M^+ eta for a Gaussian eta (complex128 device tensor (V, 4, 3))."""
        eta = T.pack_spinor(self.prob, eta_canon, T.F64, T.FULL)
        T.dslash(self.prob, self.U, eta, T.MDAG, out=self.phi, ws=self.ws_dslash)
        self._have_x = False

    def _low(self, U):
        """The links U (packed FP64) packed in the inner precision."""
        return T.pack_gauge(self.prob, T.unpack_gauge(self.prob, U), self.inner, T.RECON18)

    def refresh_low(self):
        """Re-pack the low-precision copy after the FP64 links changed."""
        if self.inner != T.F64:
            self.U_low = self._low(self.U)

    def solve(self, b, U=None, tol=None, x=None):
        """X = (M^+ M)^{-1} b on links U (default: the current links)."""
        gauges = {T.F64: self.U if U is None else U}
        if self.inner != T.F64:
            gauges[self.inner] = self.U_low if U is None else self._low(U)
        own = x is None
        x = self.X if own else x
        start_zero = not (own and self.guess and self._have_x and b is self.phi)
        _, st, _ = T.cg(self.prob, gauges, b, x, x_is_zero=start_zero, tol=tol or self.tol, max_iter=self.max_iter,
                        op=T.MDAGM, inner_prec=self.inner, ws=self.ws_cg)
        if own:
            self._have_x = b is self.phi
        self.solves += 1
        self.cg_iters += st["iters"]
        return x

    def add_gradient(self, p, scale):
        """p += scale * (G_fermion + G_gauge) at the current links."""
        X = self.solve(self.phi, tol=self.md_tol)
        T.dslash(self.prob, self.U, X, T.M, out=self.Y, ws=self.ws_dslash)
        T.force(self.prob, self.U, X, self.Y, out=p, scale=scale, accumulate=True)
        if self.beta != 0.0:
            T.gauge_force(self.prob, self.U, self.beta, out=p, scale=scale, accumulate=True)

    def energies(self, p):
        """(kinetic, S_g, S_f) as Python floats."""
        k = T.momentum_norm2(self.prob, p, ws=self.ws_aux)
        plaq = T.plaquette(self.prob, self.U, ws=self.ws_aux)
        X = self.solve(self.phi, tol=self.tol)
        sf = T.dot(self.prob, self.phi, X, T.FULL, ws=self.ws_aux)
        n_plaq = 6 * self.prob.volume
        s_g = self.beta / 3.0 * (3.0 * n_plaq - float(plaq[0])) if self.beta != 0.0 else 0.0
        return 0.5 * float(k[0]), s_g, float(sf[0])

    def hamiltonian(self, p) -> float:
        return sum(self.energies(p))

    def leapfrog(self, p, n_steps: int, dt: float):
        """Integrate (U, p) in place over n_steps * dt."""
        self.add_gradient(p, -0.5 * dt)
        for i in range(n_steps):
            T.update_links(self.prob, self.U, p, dt)
            self.refresh_low()
            self.add_gradient(p, -dt if i < n_steps - 1 else -0.5 * dt)

    def trajectory(self, p, eta_canon, uniform: float, n_steps: int, dt: float) -> dict:
        """One HMC trajectory from momenta p (modified in place) and a Gaussian eta."""
        self.refresh_low()            # the links may have been set from outside
        self.set_pseudofermion(eta_canon)
        e0 = self.energies(p)
        U0 = self.U.clone()
        self.leapfrog(p, n_steps, dt)
        e1 = self.energies(p)
        dh = sum(e1) - sum(e0)
        accepted = bool(uniform < math.exp(-dh)) if dh > 0 else True
        if not accepted:
            self.U.copy_(U0)
            self.refresh_low()
        return {"dH": dh, "accepted": accepted, "H0": sum(e0), "H1": sum(e1), "energies0": e0, "energies1": e1}
