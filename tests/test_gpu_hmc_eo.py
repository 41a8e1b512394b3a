"""The even-odd pseudofermion force and the two-level 2MN HMC on the GPU against the FP64 oracle.

* tmqcd_force_eo against the oracle's even-odd force on random X_e (several
  extents, boundary phases, both link encodings; scale and accumulate);
* on 16^3 x 32: FermionAction's backward pass with the even-odd action against
  central finite differences of phi_e^+ (Mhat^+ Mhat)^{-1} phi_e along all eight
  generators of random links (the difference formed without cancellation);
* whole even-odd trajectories with the two-level 2MN integrator (same links,
  momenta, eta_e and Metropolis draw) against the oracle's trajectory, with and
  without a gauge action on the inner level, FP64 and FP32-inner solves;
* reversibility and the dt^2 scaling of the energy error of the GPU integrator;
* the Creutz equality <exp(-dH)> = 1 on a 4^4 even-odd 2MN Markov chain.
"""
import numpy as np
import pytest
import torch

from gpu_util import BC_AP, BC_TWIST, Fields, dev, host, rel
from oracle import dirac as D
from oracle import force as F
from oracle import hmc as OH
from paper_1209_5942_amd import hmc as H
from paper_1209_5942_amd import synth
from paper_1209_5942_amd import tmqcd as T

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,bc,mu", [((4, 4, 4, 4), BC_TWIST, 0.01), ((4, 2, 6, 4), BC_AP, 0.3),
                                        ((2, 2, 2, 2), BC_TWIST, 0.05), ((6, 4, 2, 8), BC_AP, 0.0)])
@pytest.mark.parametrize("recon", [T.RECON18, T.RECON12])
def test_force_eo_matches_oracle(dims, bc, mu, recon):
    print(f"\nforce_eo dims={dims} mu={mu} recon={recon}", flush=True)
    f = Fields(dims, 0.5, 301, 0.155, mu, bc)
    vh = f.prob.volume // 2
    xe = synth.gaussian_spinor(vh, 302)
    X = T.pack_spinor(f.prob, dev(xe), T.F64, T.EVEN)
    want = F.fermion_force_eo(f.U, xe, dims, f.kappa, mu, bc)
    got = host(T.force_eo(f.prob, f.gauge(T.F64, recon), X, recon=recon))
    assert rel(got, want) < 1e-12
    p = synth.gaussian_momenta(f.prob.volume, 303)
    pd = dev(p)
    T.force_eo(f.prob, f.gauge(T.F64, recon), X, recon=recon, out=pd, scale=-0.7, accumulate=True)
    assert rel(host(pd), p - 0.7 * want) < 1e-13


@pytest.mark.timeout(900)
def test_force_eo_backward_vs_finite_differences_16x16x16x32():
    dims, kappa, mu = (16, 16, 16, 32), 0.155, 0.01
    print(f"\nforce_eo finite differences dims={dims}", flush=True)
    f = Fields(dims, 0.4, 311, kappa, mu, BC_AP)
    v = f.prob.volume
    h = H.HMC(f.prob, f.U_dev, 0.0, tol=1e-13, eo=True)
    phi = synth.gaussian_spinor(v // 2, 312)
    h.phi = T.pack_spinor(f.prob, dev(phi), T.F64, T.EVEN)
    omega = torch.zeros((v, 4, 8), dtype=torch.float64, device="cuda", requires_grad=True)
    s = H.FermionAction.apply(omega, h)
    s.backward()
    G = host(omega.grad)
    # the backward pass equals the oracle's even-odd force on the same X_e
    X = host(T.unpack_spinor(f.prob, h.solve(h.phi), T.F64, T.EVEN))
    assert rel(G, F.fermion_force_eo(f.U, X, dims, kappa, mu, BC_AP)) < 1e-11
    # S_f^eo itself: phi^+ X
    sv = float(s.detach())
    assert abs(sv - np.vdot(phi, X).real) < 1e-11 * abs(sv)
    links = synth.random_link_sample(v, 32, 313)
    hstep = 1e-5
    ws = T.workspace(f.prob, T.MHATDAGMHAT, 1)
    scale = np.abs(G).max()
    worst = 0.0
    for site, m in links:
        for a in range(8):
            us = []
            for sgn in (1, -1):
                p = torch.zeros((v, 4, 8), dtype=torch.float64, device="cuda")
                p[site, m, a] = sgn
                u = f.gauge(T.F64, 0).clone()
                T.update_links(f.prob, u, p, hstep)
                us.append(u)
            xp = h.solve(h.phi, U=us[0], x=torch.empty_like(h.X))
            xm = h.solve(h.phi, U=us[1], x=torch.empty_like(h.X))
            am = T.unpack_spinor(f.prob, T.dslash(f.prob, us[1], xm, T.MHATDAGMHAT, ws=ws), T.F64, T.EVEN)
            ap = T.unpack_spinor(f.prob, T.dslash(f.prob, us[0], xm, T.MHATDAGMHAT, ws=ws), T.F64, T.EVEN)
            xpc = T.unpack_spinor(f.prob, xp, T.F64, T.EVEN)
            diff = torch.vdot(xpc.reshape(-1), (am - ap).reshape(-1)).real.item()
            worst = max(worst, abs(diff / (2 * hstep) - G[site, m, a]) / scale)
    assert worst < 1e-7, worst


@pytest.mark.parametrize("beta,n_inner,inner", [(5.0, 1, T.F64), (5.0, 3, T.F64), (0.0, 1, T.F64),
                                                (5.0, 2, T.F32)])
def test_eo_2mn_trajectory_matches_oracle(beta, n_inner, inner):
    dims, kappa, mu = (4, 2, 2, 4), 0.155, 0.01
    print(f"\neo 2MN trajectory beta={beta} n_inner={n_inner} inner_prec={inner}", flush=True)
    f = Fields(dims, 0.4, 321, kappa, mu, BC_AP)
    p = synth.gaussian_momenta(f.prob.volume, 322)
    eta = synth.gaussian_spinor(f.prob.volume // 2, 323)
    n, dt = 4, 0.125
    want = OH.trajectory_eo(f.U, p, eta, 0.5, dims, kappa, mu, BC_AP, beta, n, dt, n_inner)
    h = H.HMC(f.prob, f.U_dev, beta, tol=1e-14, inner_prec=inner, eo=True)
    pd = dev(p)
    out = h.trajectory(pd, dev(eta), 0.5, n, dt, integrator="2mn", n_inner=n_inner)
    assert abs(out["H0"] - want["H0"]) < 1e-10 * abs(want["H0"])
    assert abs(out["dH"] - want["dH"]) < 1e-8, (out["dH"], want["dH"])
    assert out["accepted"] == want["accepted"]
    assert np.abs(host(pd) - want["p_proposed"]).max() < 1e-9
    got_u = host(T.unpack_gauge(f.prob, h.U))
    assert np.abs(got_u - (want["U_proposed"] if out["accepted"] else f.U)).max() < 1e-10
    # fermion solves: one per force (adjacent kicks merged) plus two for the energies
    assert h.solves == 2 * n + 1 + 2


def test_eo_2mn_reversible_and_second_order():
    dims, kappa, mu, beta = (4, 4, 4, 4), 0.155, 0.01, 5.6
    print(f"\neo 2MN reversibility dims={dims}", flush=True)
    f = Fields(dims, 0.4, 331, kappa, mu, BC_AP)
    p = synth.gaussian_momenta(f.prob.volume, 332)
    eta = synth.gaussian_spinor(f.prob.volume // 2, 333)
    h = H.HMC(f.prob, f.U_dev, beta, tol=1e-13, eo=True)
    h.set_pseudofermion(dev(eta))
    pd = dev(p)
    h.omelyan(pd, 5, 0.1, 2)
    pd.neg_()
    h.omelyan(pd, 5, 0.1, 2)
    assert np.abs(host(T.unpack_gauge(f.prob, h.U)) - f.U).max() < 1e-10
    assert np.abs(-host(pd) - p).max() < 1e-9
    dh = []
    for n in (4, 8):
        h2 = H.HMC(f.prob, f.U_dev, beta, tol=1e-13, eo=True)
        h2.set_pseudofermion(dev(eta))
        q = dev(p)
        h0 = h2.hamiltonian(q)
        h2.omelyan(q, n, 1.0 / n, 2)
        dh.append(h2.hamiltonian(q) - h0)
    assert 3.0 < abs(dh[0] / dh[1]) < 5.5, dh


@pytest.mark.timeout(600)
def test_creutz_equality_eo_2mn_4x4x4x4():
    """<exp(-dH)> = 1 for the even-odd action and the two-level 2MN integrator on a 4^4 chain
    (beta 5.5, kappa 0.15, mu 0.01, tau 0.5 in 4 outer steps of 2 inner steps) after 40 burn-in
    trajectories, averaged over 160 more."""
    dims = (4, 4, 4, 4)
    prob = T.Problem(dims, 0.15, 0.01, BC_AP)
    h = H.HMC(prob, dev(synth.random_links(dims, 0.3, 621).reshape(-1, 4, 3, 3)), beta=5.5, tol=1e-12,
              md_tol=1e-10, eo=True)
    rng = np.random.default_rng(622)
    dh, acc = [], 0
    for k in range(200):
        p = dev(synth.gaussian_momenta(prob.volume, 30000 + k))
        eta = dev(synth.gaussian_spinor(prob.volume // 2, 40000 + k))
        out = h.trajectory(p, eta, float(rng.random()), 4, 0.125, integrator="2mn", n_inner=2)
        if k >= 40:
            dh.append(out["dH"])
            acc += int(out["accepted"])
    e = np.exp(-np.array(dh))
    mean, err = e.mean(), e.std(ddof=1) / np.sqrt(len(e))
    print(f"eo 2MN Creutz: <exp(-dH)> = {mean:.4f} +- {err:.4f}, acceptance {acc / len(dh):.3f}", flush=True)
    assert acc / len(dh) > 0.5
    assert err < 0.05
    assert abs(mean - 1.0) < 4 * err, (mean, err)
