"""GPU HMC pieces against the FP64 oracle, and the fermion force against finite differences.

* Wilson gauge force, plaquette sum, momentum norm, spinor inner product and
  the exponential link update compared with the oracle on small lattices;
* a whole leapfrog trajectory (same links, momenta, eta and Metropolis draw)
  compared with the oracle's trajectory: dH and the proposed links;
* reversibility of the GPU leapfrog;
* the Creutz equality <exp(-dH)> = 1 on a 4^4 Markov chain after burn-in;
* on 16^3 x 32 (eps 0.4, kappa 0.155, mu 0.01, Gaussian phi): the gradient
  returned by FermionAction's backward pass (the force kernel) against central
  finite differences along all eight generators on 64 random links, with the
  difference S(U+) - S(U-) formed without cancellation as X+^+ (A- - A+) X-.
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


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 2, 6, 4), (2, 2, 2, 2)])
def test_gauge_force_plaquette_and_norms(dims):
    f = Fields(dims, 0.6, 201, 0.155, 0.01, BC_TWIST)
    g = f.gauge(T.F64, 0)
    got = host(T.gauge_force(f.prob, g, 5.6))
    assert rel(got, F.gauge_force(f.U, dims, 5.6)) < 1e-12
    # accumulate with a scale: p + (-0.3) G
    p = synth.gaussian_momenta(f.prob.volume, 202)
    pd = dev(p)
    T.gauge_force(f.prob, g, 5.6, out=pd, scale=-0.3, accumulate=True)
    assert rel(host(pd), p - 0.3 * F.gauge_force(f.U, dims, 5.6)) < 1e-13
    assert abs(float(T.plaquette(f.prob, g)[0]) - F.plaquette_sum(f.U, dims)) < 1e-12 * 18 * f.prob.volume
    assert float(T.momentum_norm2(f.prob, dev(p))[0]) == pytest.approx(float(np.sum(p * p)), rel=1e-13)
    x, y = synth.gaussian_spinor(f.prob.volume, 203), synth.gaussian_spinor(f.prob.volume, 204)
    d = host(T.dot(f.prob, T.pack_spinor(f.prob, dev(x)), T.pack_spinor(f.prob, dev(y))))
    want = np.vdot(x, y)
    assert abs(complex(d[0], d[1]) - want) < 1e-12 * abs(want)


@pytest.mark.parametrize("dt", [0.05, 1.7])
def test_update_links_matches_oracle_exponential(dt):
    dims = (4, 4, 2, 4)
    f = Fields(dims, 0.5, 211, 0.155, 0.01, BC_AP)
    p = synth.gaussian_momenta(f.prob.volume, 212)
    g = f.gauge(T.F64, 0).clone()
    T.update_links(f.prob, g, dev(p), dt)
    got = host(T.unpack_gauge(f.prob, g))
    want = OH.su3_exp(p, dt) @ f.U
    assert np.abs(got - want).max() < 1e-13
    np.testing.assert_allclose(np.linalg.det(got), 1.0, atol=1e-13)


@pytest.mark.parametrize("inner", [T.F64, T.F32])
def test_trajectory_matches_oracle(inner):
    """Whole trajectory against the oracle, with FP64 solves and with FP32-inner defect correction."""
    dims, kappa, mu, beta = (2, 2, 2, 4), 0.155, 0.01, 5.0
    f = Fields(dims, 0.4, 221, kappa, mu, BC_AP)
    p = synth.gaussian_momenta(f.prob.volume, 222)
    eta = synth.gaussian_spinor(f.prob.volume, 223)
    n, dt = 8, 0.125
    want = OH.trajectory(f.U, p, eta, 0.5, dims, kappa, mu, BC_AP, beta, n, dt)
    h = H.HMC(f.prob, f.U_dev, beta, tol=1e-14, inner_prec=inner)
    pd = dev(p)
    out = h.trajectory(pd, dev(eta), 0.5, n, dt)
    assert abs(out["dH"] - want["dH"]) < 1e-8
    assert abs(out["H0"] - want["H0"]) < 1e-9 * abs(want["H0"])
    assert out["accepted"] == want["accepted"]
    if out["accepted"]:
        assert np.abs(host(T.unpack_gauge(f.prob, h.U)) - want["U_proposed"]).max() < 1e-10
    assert np.abs(host(pd) - want["p_proposed"]).max() < 1e-9


def test_leapfrog_reversible_and_second_order():
    dims, kappa, mu, beta = (4, 4, 4, 4), 0.155, 0.01, 5.6
    f = Fields(dims, 0.4, 231, kappa, mu, BC_AP)
    p = synth.gaussian_momenta(f.prob.volume, 232)
    eta = synth.gaussian_spinor(f.prob.volume, 233)
    h = H.HMC(f.prob, f.U_dev, beta, tol=1e-13)
    h.set_pseudofermion(dev(eta))
    pd = dev(p)
    h.leapfrog(pd, 10, 0.05)
    pd.neg_()
    h.leapfrog(pd, 10, 0.05)
    assert np.abs(host(T.unpack_gauge(f.prob, h.U)) - f.U).max() < 1e-10
    assert np.abs(-host(pd) - p).max() < 1e-9
    dh = []
    for n in (10, 20):
        h2 = H.HMC(f.prob, f.U_dev, beta, tol=1e-13)
        h2.set_pseudofermion(dev(eta))
        q = dev(p)
        h0 = h2.hamiltonian(q)
        h2.leapfrog(q, n, 0.5 / n)
        dh.append(h2.hamiltonian(q) - h0)
    assert 3.0 < abs(dh[0] / dh[1]) < 5.5, dh


@pytest.mark.timeout(900)
def test_fermion_force_vs_finite_differences_16x16x16x32():
    dims, kappa, mu = (16, 16, 16, 32), 0.155, 0.01
    f = Fields(dims, 0.4, 241, kappa, mu, BC_AP)
    v = f.prob.volume
    h = H.HMC(f.prob, f.U_dev, 0.0, tol=1e-13)
    phi = synth.gaussian_spinor(v, 242)
    h.phi = T.pack_spinor(f.prob, dev(phi))
    omega = torch.zeros((v, 4, 8), dtype=torch.float64, device="cuda", requires_grad=True)
    s = H.FermionAction.apply(omega, h)
    s.backward()
    G = host(omega.grad)
    # the backward pass equals the oracle's force formula on the same X, Y = M X
    X = host(T.unpack_spinor(f.prob, h.solve(h.phi)))
    Y = D.apply_M(f.U, X, dims, kappa, mu, BC_AP)
    assert rel(G, F.fermion_force(f.U, X, Y, dims, kappa, BC_AP)) < 1e-11
    # and central finite differences along every generator of 64 random links
    links = synth.random_link_sample(v, 64, 243)
    hstep = 1e-5
    ws = T.workspace(f.prob, T.MDAGM, 1)
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
            am = T.unpack_spinor(f.prob, T.dslash(f.prob, us[1], xm, T.MDAGM, ws=ws))
            ap = T.unpack_spinor(f.prob, T.dslash(f.prob, us[0], xm, T.MDAGM, ws=ws))
            diff = torch.vdot(T.unpack_spinor(f.prob, xp).reshape(-1), (am - ap).reshape(-1)).real.item()
            err = abs(diff / (2 * hstep) - G[site, m, a]) / scale
            worst = max(worst, err)
    assert worst < 1e-7, worst


@pytest.mark.timeout(600)
def test_creutz_equality_in_equilibrium_4x4x4x4():
    """<exp(-dH)> = 1 holds for a reversible, area-preserving integrator when (U, p, phi) follow
    exp(-H): a 4^4 chain (beta 5.5, kappa 0.15, mu 0.01, tau 0.5 in 10 steps) after 40 burn-in
    trajectories, averaged over 160 more."""
    dims = (4, 4, 4, 4)
    prob = T.Problem(dims, 0.15, 0.01, BC_AP)
    h = H.HMC(prob, dev(synth.random_links(dims, 0.3, 601).reshape(-1, 4, 3, 3)), beta=5.5, tol=1e-12,
              md_tol=1e-10)
    rng = np.random.default_rng(602)
    dh, acc = [], 0
    for k in range(200):
        p = dev(synth.gaussian_momenta(prob.volume, 10000 + k))
        eta = dev(synth.gaussian_spinor(prob.volume, 20000 + k))
        out = h.trajectory(p, eta, float(rng.random()), 10, 0.05)
        if k >= 40:
            dh.append(out["dH"])
            acc += int(out["accepted"])
    e = np.exp(-np.array(dh))
    mean, err = e.mean(), e.std(ddof=1) / np.sqrt(len(e))
    assert acc / len(dh) > 0.5
    assert err < 0.05
    assert abs(mean - 1.0) < 4 * err, (mean, err)


def test_mixed_precision_trajectory_equals_fp64_16x16x16x32():
    """FP32-inner solves reach the same FP64 tolerances: the trajectory's dH and links agree with FP64 solves,
    also when every solve starts from the previous solution (which must save iterations)."""
    dims = (16, 16, 16, 32)
    f = Fields(dims, 0.4, 611, 0.155, 0.01, BC_AP)
    p = synth.gaussian_momenta(f.prob.volume, 612)
    eta = synth.gaussian_spinor(f.prob.volume, 613)
    out, links, iters = [], [], []
    for inner, guess in ((T.F64, False), (T.F32, False), (T.F32, True)):
        h = H.HMC(f.prob, f.U_dev, 0.0, tol=1e-12, md_tol=1e-11, inner_prec=inner, guess=guess)
        out.append(h.trajectory(dev(p), dev(eta), 0.0, 4, 0.05))
        links.append(host(T.unpack_gauge(f.prob, h.U)))
        iters.append(h.cg_iters)
    for k in (1, 2):   # FP32-inner solves, from zero and from the previous solution
        assert abs(out[0]["H0"] - out[k]["H0"]) < 1e-9 * abs(out[0]["H0"])
        assert abs(out[0]["dH"] - out[k]["dH"]) < 1e-6, (out[0]["dH"], out[k]["dH"])
        assert np.abs(links[0] - links[k]).max() < 1e-9
    assert iters[2] < iters[1]


@pytest.mark.parametrize("eo", [False, True])
def test_fermion_action_backward_keeps_its_own_links_and_solution(eo):
    """Two forwards at different omega summed, the HMC's links and solve buffer changed in
    between, then one backward: each omega receives the oracle's force at its own links
    exp(i omega.T) U with its own solution."""
    dims, kappa, mu = (4, 4, 4, 4), 0.15, 0.01
    f = Fields(dims, 0.3, 251, kappa, mu, BC_AP)
    v = f.prob.volume
    h = H.HMC(f.prob, f.U_dev, 0.0, tol=1e-13, eo=eo)
    n = v // 2 if eo else v
    h.set_pseudofermion(dev(synth.gaussian_spinor(n, 252)))
    phi = host(T.unpack_spinor(f.prob, h.phi, T.F64, h.subset))
    w2 = 0.05 * synth.gaussian_momenta(v, 253)
    om1 = torch.zeros((v, 4, 8), dtype=torch.float64, device="cuda", requires_grad=True)
    om2 = torch.tensor(w2, dtype=torch.float64, device="cuda", requires_grad=True)
    s = H.FermionAction.apply(om1, h) + H.FermionAction.apply(om2, h)
    # the state moves on before the backward pass: another solve and a link update
    h.solve(h.phi)
    T.update_links(f.prob, h.U, dev(synth.gaussian_momenta(v, 254)), 0.1)
    s.backward()
    U2 = OH.su3_exp(w2, 1.0) @ f.U.reshape(-1, 4, 3, 3)
    for om, U in ((om1, f.U.reshape(-1, 4, 3, 3)), (om2, U2)):
        if eo:
            Xe, _ = D.cg(lambda x: D.apply_MhatdagMhat(U, x, dims, kappa, mu, BC_AP), phi, 1e-14)
            want = F.fermion_force_eo(U, Xe, dims, kappa, mu, BC_AP)
        else:
            X, _ = D.cg(lambda x: D.apply_MdagM(U, x, dims, kappa, mu, BC_AP), phi, 1e-14)
            want = F.fermion_force(U, X, D.apply_M(U, X, dims, kappa, mu, BC_AP), dims, kappa, BC_AP)
        assert rel(host(om.grad), want) < 1e-10


@pytest.mark.parametrize("subset,beta,c1", [(T.FULL, 0.0, 0.0), (T.FULL, 5.5, 0.0), (T.EVEN, 3.9, -1.0 / 12.0)])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 8)])
def test_delta_h_summed_site_by_site_matches_oracle(subset, beta, c1, dims):
    """tmqcd_delta_h between two unrelated states (links, momenta, solutions) against the oracle's
    parts: 1/2 sum (p1^2 - p0^2), the gauge actions' difference (plaquettes and rectangles) and
    Re phi^+ (X1 - X0)."""
    from oracle import symanzik as S
    prob = T.Problem(dims, 0.15, 0.01, BC_AP)
    v = prob.volume
    U0 = synth.random_links(dims, 0.4, 261)
    U1 = synth.random_links(dims, 0.4, 262)
    p0, p1 = synth.gaussian_momenta(v, 263), synth.gaussian_momenta(v, 264)
    n = v if subset == T.FULL else v // 2
    phi, x0, x1 = (synth.gaussian_spinor(n, 265 + k) for k in range(3))
    pk = lambda a: T.pack_spinor(prob, dev(a), T.F64, subset)
    d = host(T.delta_h(prob, T.pack_gauge(prob, dev(U0)), T.pack_gauge(prob, dev(U1)), dev(p0), dev(p1), pk(phi),
                       pk(x0), pk(x1), subset, beta, c1))
    kin = 0.5 * (np.sum(p1 ** 2) - np.sum(p0 ** 2))
    gauge = 0.0
    if beta != 0.0:
        gauge = beta / 3.0 * ((1 - 8 * c1) * (S.plaquette_sum(U0, dims) - S.plaquette_sum(U1, dims))
                              + c1 * (S.rectangle_sum(U0, dims) - S.rectangle_sum(U1, dims)))
    ferm = float(np.vdot(phi, x1 - x0).real)
    for got, want in ((d[1], kin), (d[2], gauge), (d[3], ferm), (d[0], kin + gauge + ferm)):
        assert abs(got - want) <= 1e-12 * max(1.0, abs(kin) + abs(gauge) + abs(ferm)), (got, want)
