"""Hybrid Monte-Carlo and the differentiable pseudofermion action on the HIP library.

Paper, ensemble-generation section: H = 1/2 P^2 + S_g + S_f with momenta P
conjugate to U, evolved with a symplectic integrator and followed by a
Metropolis step.  Here:

* S_f = phi^+ (M^+ M)^{-1} phi on the full lattice, phi = M^+ eta, or (eo=True)
  the even-odd action S_f = phi_e^+ (Mhat^+ Mhat)^{-1} phi_e, phi_e = Mhat^+ eta_e,
  with the pseudofermion on even sites only; eta Gaussian (random numbers are
  inputs);
* S_g = (beta/3) sum_x [c0 sum_{mu<nu} (3 - Re Tr P_mu_nu) + c1 sum_{mu!=nu}
  (3 - Re Tr R_mu_nu)], c0 = 1 - 8 c1: the paper's tree-level Symanzik action
  (c1 = -1/12; c1 = 0, the default, is the Wilson plaquette action);
* leapfrog: half momentum step, n times (link step, momentum step), the last
  momentum step a half step; U <- exp(i dt p^a T^a) U; p <- p - dt G;
* the paper's production integrator, second-order minimal norm (2MN, Omelyan)
  on two timescales: per outer step dt the fermion force kicks with weights
  lam, 1 - 2 lam, lam around two inner integrations over dt/2, each n_inner
  2MN steps of the gauge force (Sexton-Weingarten nesting); lam = LAMBDA_2MN.
  Adjacent kicks at the same links are merged, so an outer step costs two
  fermion forces (one solve each);
* Metropolis: accept with probability min(1, exp(-(H' - H))), with H' - H summed site
  by site in FP64 on the device (tmqcd_delta_h) from both states.

Every step runs in libtmqcd kernels (CG, force, gauge force, link update,
reductions); torch provides device buffers and the copies that keep the
rejected configuration.  :class:`FermionAction` exposes S_f to autograd: its
backward pass is the fermion-force kernel.
"""
from __future__ import annotations

import math

import torch

from . import tmqcd as T

# Omelyan, Mryglod and Folk's minimal-norm coefficient of the second-order scheme
LAMBDA_2MN = 0.1931833275037836


class FermionAction(torch.autograd.Function):
    """S_f(omega) = phi^+ (M^+ M)^{-1} phi (or the even-odd phi_e^+ (Mhat^+ Mhat)^{-1} phi_e
    when the HMC state has eo=True) at links exp(i omega^a T^a) U.

    forward(omega, ctx_obj) with omega a float64 device tensor (V, 4, 8) and
    ctx_obj a :class:`HMC`; returns a 0-dim float64 tensor.  The backward pass
    returns the fermion force G evaluated at the links exp(i omega.T) U: the
    derivative of S_f along left translations there, equal to dS_f/domega at
    omega = 0 (where HMC evaluates it).
    """

    @staticmethod
    def forward(ctx, omega, h: "HMC"):
        # The backward pass needs the links and the solution of this call: both are kept
        # in buffers of their own, since the HMC state's links change in place and its
        # solve buffer is reused by every later solve.
        U = h.U.clone()
        if bool(torch.any(omega != 0)):
            T.update_links(h.prob, U, omega, 1.0)
        X = h.solve(h.phi, U, x=torch.empty_like(h.X))
        s = T.dot(h.prob, h.phi, X, h.subset, ws=h.ws_aux)
        ctx.h, ctx.U, ctx.X = h, U, X
        return s[0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        h = ctx.h
        if h.eo:
            return T.force_eo(h.prob, ctx.U, ctx.X, scale=float(grad_out), ws=h.ws_force), None
        # Y = M X is formed by the force call itself, in its workspace
        return T.force(h.prob, ctx.U, ctx.X, None, scale=float(grad_out), ws=h.ws_force), None


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

    eo: the even-odd pseudofermion action (solves on Mhat^+ Mhat over half the
    sites, the force of tmqcd_force_eo) in place of the full-lattice one.

    c1: rectangle coefficient of the tree-level Symanzik gauge action.
    """

    def __init__(self, prob: T.Problem, U_canon, beta: float, tol: float = 1e-12, max_iter: int = 20000,
                 md_tol: float | None = None, inner_prec: int = T.F64, guess: bool = False, eo: bool = False,
                 c1: float = 0.0):
        self.prob = prob
        self.beta = float(beta)
        self.c1 = float(c1)
        self.tol = tol                      # solves that enter H (acceptance)
        self.md_tol = md_tol or tol         # solves that enter the force
        self.max_iter = max_iter
        self.inner = inner_prec
        self.guess = guess
        self.eo = eo
        self.op = T.MHATDAGMHAT if eo else T.MDAGM
        self.subset = T.EVEN if eo else T.FULL
        self._have_x = False      # self.X holds a solution for the current phi
        self.U = T.pack_gauge(prob, U_canon, T.F64, T.RECON18)
        self.U_low = None
        self.refresh_low()
        dev = self.U.device
        fb = T.spinor_bytes(prob, T.F64, self.subset)
        self.ws_cg = T.workspace(prob, self.op, 1 | (1 << inner_prec))
        self.ws_dslash = T.workspace(prob, self.op, 1)
        self.ws_aux = T.aux_workspace(prob)
        self.ws_force = T._bytes(T.force_eo_workspace_bytes(prob) if eo else T.force_workspace_bytes(prob), dev)
        self.ws_gauge = T._bytes(T.gauge_force_tlsym_workspace_bytes(prob), dev) if c1 != 0.0 else None
        self.X = torch.empty(fb, dtype=torch.uint8, device=dev)
        self.phi = torch.empty(fb, dtype=torch.uint8, device=dev)
        self.solves = 0
        self.cg_iters = 0

    # --------------------------------------------------------------- pieces ---
    def set_pseudofermion(self, eta_canon):
        """phi = M^+ eta for a Gaussian eta (complex128 device tensor (V, 4, 3)); with eo,
        phi_e = Mhat^+ eta_e for eta_e on the even sites ((V/2, 4, 3))."""
        eta = T.pack_spinor(self.prob, eta_canon, T.F64, self.subset)
        T.dslash(self.prob, self.U, eta, T.MHATDAG if self.eo else T.MDAG, out=self.phi, ws=self.ws_dslash)
        self._have_x = False

    def _low(self, U):
        """The links U (packed FP64) packed in the inner precision."""
        return T.pack_gauge(self.prob, T.unpack_gauge(self.prob, U), self.inner, T.RECON18)

    def refresh_low(self):
        """Re-pack the low-precision copy after the FP64 links changed."""
        if self.inner != T.F64:
            self.U_low = self._low(self.U)

    def solve(self, b, U=None, tol=None, x=None):
        """X = (M^+ M)^{-1} b (with eo, (Mhat^+ Mhat)^{-1} b_e) on links U (default: the current links)."""
        gauges = {T.F64: self.U if U is None else U}
        if self.inner != T.F64:
            gauges[self.inner] = self.U_low if U is None else self._low(U)
        own = x is None
        x = self.X if own else x
        start_zero = not (own and self.guess and self._have_x and b is self.phi)
        _, st, _ = T.cg(self.prob, gauges, b, x, x_is_zero=start_zero, tol=tol or self.tol, max_iter=self.max_iter,
                        op=self.op, inner_prec=self.inner, ws=self.ws_cg)
        if own:
            self._have_x = b is self.phi
        self.solves += 1
        self.cg_iters += st["iters"]
        return x

    def add_fermion_gradient(self, p, scale):
        """p += scale * G_fermion at the current links (one solve)."""
        X = self.solve(self.phi, tol=self.md_tol)
        if self.eo:
            T.force_eo(self.prob, self.U, X, out=p, scale=scale, accumulate=True, ws=self.ws_force)
        else:
            T.force(self.prob, self.U, X, None, out=p, scale=scale, accumulate=True, ws=self.ws_force)

    def add_gauge_gradient(self, p, scale):
        """p += scale * G_gauge at the current links."""
        if self.beta == 0.0:
            return
        if self.c1 != 0.0:
            T.gauge_force_tlsym(self.prob, self.U, self.beta, self.c1, out=p, scale=scale, accumulate=True,
                                ws=self.ws_gauge)
        else:
            T.gauge_force(self.prob, self.U, self.beta, out=p, scale=scale, accumulate=True)

    def add_gradient(self, p, scale):
        """p += scale * (G_fermion + G_gauge) at the current links."""
        self.add_fermion_gradient(p, scale)
        self.add_gauge_gradient(p, scale)

    def energies(self, p):
        """(kinetic, S_g, S_f) as Python floats."""
        k = T.momentum_norm2(self.prob, p, ws=self.ws_aux)
        plaq = T.plaquette(self.prob, self.U, ws=self.ws_aux)
        X = self.solve(self.phi, tol=self.tol)
        sf = T.dot(self.prob, self.phi, X, self.subset, ws=self.ws_aux)
        n_plaq = 6 * self.prob.volume
        s_g = 0.0
        if self.beta != 0.0:
            c0 = 1.0 - 8.0 * self.c1
            s_g = self.beta / 3.0 * c0 * (3.0 * n_plaq - float(plaq[0]))
            if self.c1 != 0.0:
                rect = T.rectangle(self.prob, self.U, ws=self.ws_aux)
                s_g += self.beta / 3.0 * self.c1 * (3.0 * 2 * n_plaq - float(rect[0]))
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

    def _inner(self, p, tau: float, n_inner: int, lam: float):
        """The inner level of 2MN over tau: n_inner steps with the gauge force, or the
        plain link update when there is no gauge action."""
        if self.beta == 0.0:
            T.update_links(self.prob, self.U, p, tau)
        else:
            h = tau / n_inner
            self.add_gauge_gradient(p, -lam * h)
            for j in range(n_inner):
                T.update_links(self.prob, self.U, p, 0.5 * h)
                self.add_gauge_gradient(p, -(1.0 - 2.0 * lam) * h)
                T.update_links(self.prob, self.U, p, 0.5 * h)
                self.add_gauge_gradient(p, -(2.0 * lam if j < n_inner - 1 else lam) * h)
        self.refresh_low()

    def omelyan(self, p, n_outer: int, dt: float, n_inner: int = 1, lam: float = LAMBDA_2MN):
        """Integrate (U, p) in place over n_outer * dt with the two-level 2MN scheme
        (fermion force on the outer scale, gauge force on the inner one)."""
        self.add_fermion_gradient(p, -lam * dt)
        for i in range(n_outer):
            self._inner(p, 0.5 * dt, n_inner, lam)
            self.add_fermion_gradient(p, -(1.0 - 2.0 * lam) * dt)
            self._inner(p, 0.5 * dt, n_inner, lam)
            self.add_fermion_gradient(p, -(2.0 * lam if i < n_outer - 1 else lam) * dt)

    def trajectory(self, p, eta_canon, uniform: float, n_steps: int, dt: float, integrator: str = "leapfrog",
                   n_inner: int = 1) -> dict:
        """One HMC trajectory from momenta p (modified in place) and a Gaussian eta.

        integrator "leapfrog" (n_steps steps) or "2mn" (n_steps outer steps of the
        two-level scheme, n_inner inner steps per half outer step)."""
        if integrator not in ("leapfrog", "2mn"):
            raise ValueError(f"unknown integrator {integrator!r}")
        self.refresh_low()            # the links may have been set from outside
        self.set_pseudofermion(eta_canon)
        e0 = self.energies(p)
        U0, p0, X0 = self.U.clone(), p.clone(), self.X.clone()
        if integrator == "leapfrog":
            self.leapfrog(p, n_steps, dt)
        else:
            self.omelyan(p, n_steps, dt, n_inner)
        e1 = self.energies(p)
        # dH summed site by site in FP64 on the device, from both states' links, momenta and solutions
        d = T.delta_h(self.prob, U0, self.U, p0, p, self.phi, X0, self.X, self.subset, self.beta, self.c1,
                      ws=self.ws_aux)
        dh = float(d[0])
        accepted = bool(uniform < math.exp(-dh)) if dh > 0 else True
        if not accepted:
            self.U.copy_(U0)
            self.refresh_low()
        return {"dH": dh, "accepted": accepted, "H0": sum(e0), "H1": sum(e1), "energies0": e0, "energies1": e1,
                "dH_parts": [float(v) for v in d[1:].cpu()], "dH_from_totals": sum(e1) - sum(e0)}
