"""Pins for the oracle's even-odd pseudofermion action, its force, and the two-level 2MN integrator (no GPU).

* The even-odd force against central finite differences of S_f^eo along all
  eight generators, the difference formed without cancellation as
  X+^dag (A- - A+) X- with A = Mhat^dag Mhat.
* phi_e = Mhat^dag eta_e gives S_f^eo = eta_e^dag eta_e exactly.
* 2MN: time reversibility, an energy error shrinking as dt^2 (for one and for
  two timescales), and the pure link update when there is no inner force.
"""
import numpy as np
import pytest

from oracle import dirac as D
from oracle import force as F
from oracle import hmc as H
from paper_1209_5942_amd import synth

BC = (1, 1, 1, -1)
BC_TWIST = (np.exp(0.3j), 1.0, np.exp(-0.4j), -1.0)


def _perturb(U, site, mu, a, h):
    u = U.copy()
    u[site, mu] = H.su3_exp(h * np.eye(8)[a], 1.0) @ U[site, mu]
    return u


def _solve_eo(U, phi_e, dims, kappa, mu, bc):
    x, _ = D.cg(lambda v: D.apply_MhatdagMhat(U, v, dims, kappa, mu, bc), phi_e, 1e-14)
    return x


SITES = [(0, 0), (5, 1), (17, 2), (63, 3), (2, 3), (9, 0)]


@pytest.mark.parametrize("bc,mu", [(BC, 0.01), (BC_TWIST, 0.2)])
def test_eo_force_vs_finite_differences(bc, mu, sites=SITES):
    dims, kappa = (4, 2, 2, 4), 0.15
    vh = int(np.prod(dims)) // 2
    U = synth.random_links(dims, 0.4, 81)
    phi = synth.gaussian_spinor(vh, 82)
    X = _solve_eo(U, phi, dims, kappa, mu, bc)
    G = F.fermion_force_eo(U, X, dims, kappa, mu, bc)
    h = 1e-5
    A = lambda u, v: D.apply_MhatdagMhat(u, v, dims, kappa, mu, bc)
    # links from even and from odd sites, every direction
    for site, m in sites:
        for a in range(8):
            up, um = _perturb(U, site, m, a, h), _perturb(U, site, m, a, -h)
            xp, xm = _solve_eo(up, phi, dims, kappa, mu, bc), _solve_eo(um, phi, dims, kappa, mu, bc)
            fd = np.vdot(xp, A(um, xm) - A(up, xm)).real / (2 * h)
            assert abs(fd - G[site, m, a]) < 2e-8 * max(1.0, np.abs(G).max()), (site, m, a, fd, G[site, m, a])


def test_eo_action_of_mhatdag_eta_is_eta_norm():
    dims, kappa, mu = (4, 4, 2, 2), 0.155, 0.03
    vh = int(np.prod(dims)) // 2
    U = synth.random_links(dims, 0.4, 83)
    eta = synth.gaussian_spinor(vh, 84)
    phi = D.apply_Mhatdag(U, eta, dims, kappa, mu, BC)
    s, _ = F.fermion_action_eo(U, phi, dims, kappa, mu, BC)
    assert abs(s - np.vdot(eta, eta).real) < 1e-10 * np.vdot(eta, eta).real


def _eo_setup(seed=91, beta=5.0):
    dims, kappa, mu = (4, 2, 2, 4), 0.155, 0.01
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, seed)
    p = synth.gaussian_momenta(v, seed + 1)
    eta = synth.gaussian_spinor(v // 2, seed + 2)
    phi = D.apply_Mhatdag(U, eta, dims, kappa, mu, BC)
    act = H._ActionEO(dims, kappa, mu, BC, beta, 1e-14)
    return dims, kappa, mu, beta, U, p, phi, act


@pytest.mark.parametrize("n_inner", [1, 3])
def test_omelyan_reversible(n_inner):
    dims, kappa, mu, beta, U, p, phi, act = _eo_setup()
    go = lambda u: act.fermion_gradient(u, phi)
    u1, p1 = H.omelyan(U, p, go, act.gauge_gradient, 3, 0.1, n_inner)
    u2, p2 = H.omelyan(u1, -p1, go, act.gauge_gradient, 3, 0.1, n_inner)
    assert np.abs(u2 - U).max() < 1e-11
    assert np.abs(-p2 - p).max() < 1e-10


@pytest.mark.parametrize("n_inner", [1, 3])
def test_omelyan_energy_error_is_second_order(n_inner):
    dims, kappa, mu, beta, U, p, phi, act = _eo_setup()
    go = lambda u: act.fermion_gradient(u, phi)
    h0 = H.hamiltonian_eo(U, p, phi, dims, kappa, mu, BC, beta)
    dh = []
    for n in (4, 8):
        u1, p1 = H.omelyan(U, p, go, act.gauge_gradient, n, 0.4 / n, n_inner)
        dh.append(H.hamiltonian_eo(u1, p1, phi, dims, kappa, mu, BC, beta) - h0)
    assert 3.0 < abs(dh[0] / dh[1]) < 5.5, dh


def test_omelyan_without_inner_force_moves_links_by_the_exponential():
    dims, kappa, mu, beta, U, p, phi, act = _eo_setup(beta=0.0)
    zero = lambda u: np.zeros(u.shape[:2] + (8,))
    u1, p1 = H.omelyan(U, p, zero, None, 3, 0.2)
    np.testing.assert_allclose(p1, p, atol=0)
    np.testing.assert_allclose(u1, H.su3_exp(p, 0.6) @ U, atol=1e-13)


def test_eo_trajectory_metropolis_and_proposal():
    dims, kappa, mu, beta = (4, 2, 2, 4), 0.155, 0.01, 5.0
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, 95)
    p = synth.gaussian_momenta(v, 96)
    eta = synth.gaussian_spinor(v // 2, 97)
    out = H.trajectory_eo(U, p, eta, 0.3, dims, kappa, mu, BC, beta, 4, 0.1, 2)
    assert abs(out["H0"] - (0.5 * np.sum(p * p) + np.vdot(eta, eta).real + F.gauge_action(U, dims, beta))) < 1e-8
    assert out["accepted"] == (0.3 < np.exp(-out["dH"]))
    assert abs(out["dH"]) < 0.5


def test_2mn_lambda_is_the_minimal_norm_value():
    # Omelyan, Mryglod and Folk's closed form of the second-order minimal-norm coefficient
    c = (2.0 * np.sqrt(326.0) + 36.0) ** (1.0 / 3.0)
    assert abs(H.LAMBDA_2MN - (0.5 - c / 12.0 + 1.0 / (6.0 * c))) < 1e-15


def test_omelyan_with_symanzik_inner_force_is_reversible_and_second_order():
    dims, kappa, mu, beta, U, p, phi, _ = _eo_setup()
    act = H._ActionEO(dims, kappa, mu, BC, beta, 1e-14, c1=-1.0 / 12.0)
    go = lambda u: act.fermion_gradient(u, phi)
    u1, p1 = H.omelyan(U, p, go, act.gauge_gradient, 2, 0.1, 2)
    u2, p2 = H.omelyan(u1, -p1, go, act.gauge_gradient, 2, 0.1, 2)
    assert np.abs(u2 - U).max() < 1e-11
    assert np.abs(-p2 - p).max() < 1e-10
    h0 = H.hamiltonian_eo(U, p, phi, dims, kappa, mu, BC, beta, c1=-1.0 / 12.0)
    dh = []
    for n in (4, 8):
        u1, p1 = H.omelyan(U, p, go, act.gauge_gradient, n, 0.4 / n, 2)
        dh.append(H.hamiltonian_eo(u1, p1, phi, dims, kappa, mu, BC, beta, c1=-1.0 / 12.0) - h0)
    assert 3.0 < abs(dh[0] / dh[1]) < 5.5, dh
