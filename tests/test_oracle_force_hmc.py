"""Pins for the oracle's fermion force, gauge force and leapfrog HMC (no GPU).

* Gradients against central finite differences along all eight su(3)
  generators.  For S_f the difference S(U+) - S(U-) is formed without
  cancellation as X+^dag (A- - A+) X-, with X+- = A+-^{-1} phi and A = M^dag M.
* The fermion force transforms in the adjoint under a gauge transformation.
* Leapfrog: time reversibility, energy error shrinking as dt^2, and exact
  equality of the phi = M^dag eta action with eta^dag eta.
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


def _solve(U, phi, dims, kappa, mu, bc):
    x, _ = D.cg(lambda v: D.apply_MdagM(U, v, dims, kappa, mu, bc), phi, 1e-14)
    return x


@pytest.mark.parametrize("bc", [BC, BC_TWIST])
def test_fermion_force_vs_finite_differences(bc):
    dims, kappa, mu = (4, 2, 2, 4), 0.15, 0.01
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, 51)
    phi = synth.gaussian_spinor(v, 52)
    X = _solve(U, phi, dims, kappa, mu, bc)
    Y = D.apply_M(U, X, dims, kappa, mu, bc)
    G = F.fermion_force(U, X, Y, dims, kappa, bc)
    h = 1e-5
    links = [(0, 0), (5, 1), (17, 2), (63, 3)] if bc == BC else [(3, 0), (60, 3)]
    for site, m in links:
        for a in range(8):
            up, um = _perturb(U, site, m, a, h), _perturb(U, site, m, a, -h)
            xp, xm = _solve(up, phi, dims, kappa, mu, bc), _solve(um, phi, dims, kappa, mu, bc)
            diff = np.vdot(xp, D.apply_MdagM(um, xm, dims, kappa, mu, bc)
                           - D.apply_MdagM(up, xm, dims, kappa, mu, bc)).real
            fd = diff / (2 * h)
            assert abs(fd - G[site, m, a]) < 2e-8 * max(1.0, np.abs(G).max()), (site, m, a, fd, G[site, m, a])


def test_fermion_force_is_gauge_covariant():
    dims, kappa, mu = (4, 2, 2, 4), 0.15, 0.01
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, 61)
    om = synth.random_gauge_transform(v, 2.0, 62)
    X = synth.gaussian_spinor(v, 63)
    Y = D.apply_M(U, X, dims, kappa, mu, BC)
    c = D.coords(dims)
    ug = np.empty_like(U)
    for m in range(4):
        cf = c.copy()
        cf[:, m] = (cf[:, m] + 1) % dims[m]
        fwd = cf[:, 0] + dims[0] * (cf[:, 1] + dims[1] * (cf[:, 2] + dims[2] * cf[:, 3]))
        ug[:, m] = om @ U[:, m] @ om[fwd].conj().transpose(0, 2, 1)
    rot = lambda f: np.einsum("nab,nsb->nsa", om, f)
    g0 = F.fermion_force(U, X, Y, dims, kappa, BC)
    g1 = F.fermion_force(ug, rot(X), rot(Y), dims, kappa, BC)
    mat = lambda g: np.einsum("nma,aij->nmij", g, F.T_GEN)
    want = np.einsum("nab,nmbc,ndc->nmad", om, mat(g0), om.conj())
    np.testing.assert_allclose(mat(g1), want, atol=1e-12)


def test_gauge_force_vs_finite_differences():
    dims, beta = (4, 2, 2, 4), 5.6
    U = synth.random_links(dims, 0.6, 71)
    G = F.gauge_force(U, dims, beta)
    h = 1e-5
    for site, m in [(0, 0), (9, 1), (33, 2), (62, 3)]:
        for a in range(8):
            sp_ = F.gauge_action(_perturb(U, site, m, a, h), dims, beta)
            sm_ = F.gauge_action(_perturb(U, site, m, a, -h), dims, beta)
            assert abs((sp_ - sm_) / (2 * h) - G[site, m, a]) < 1e-6


def test_gauge_action_of_unit_field_and_plaquette_count():
    dims = (2, 4, 2, 4)
    U = synth.unit_links(dims)
    assert F.plaquette_sum(U, dims) == pytest.approx(3 * 6 * 64)
    assert F.gauge_action(U, dims, 5.0) == pytest.approx(0.0, abs=1e-10)


def test_pseudofermion_action_equals_eta_norm():
    # phi = M^dag eta  =>  phi^dag (M^dag M)^{-1} phi = eta^dag eta exactly
    dims, kappa, mu = (4, 2, 2, 4), 0.155, 0.01
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, 81)
    eta = synth.gaussian_spinor(v, 82)
    phi = D.apply_Mdag(U, eta, dims, kappa, mu, BC)
    s, _ = F.fermion_action(U, phi, dims, kappa, mu, BC)
    assert s == pytest.approx(np.vdot(eta, eta).real, rel=1e-12)


def test_leapfrog_reversible_and_second_order():
    dims, kappa, mu, beta = (2, 2, 2, 2), 0.155, 0.01, 5.0
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, 91)
    p = synth.gaussian_momenta(v, 92)
    eta = synth.gaussian_spinor(v, 93)
    phi = D.apply_Mdag(U, eta, dims, kappa, mu, BC)
    args = (dims, kappa, mu, BC, beta)
    u1, p1 = H.leapfrog(U, p, phi, *args, n_steps=8, dt=0.0625)
    u2, p2 = H.leapfrog(u1, -p1, phi, *args, n_steps=8, dt=0.0625)
    assert np.abs(u2 - U).max() < 1e-10
    assert np.abs(-p2 - p).max() < 1e-10
    h0 = H.hamiltonian(U, p, phi, *args)
    dh = []
    for n in (8, 16):
        un, pn = H.leapfrog(U, p, phi, *args, n_steps=n, dt=0.5 / n)
        dh.append(H.hamiltonian(un, pn, phi, *args) - h0)
    ratio = abs(dh[0] / dh[1])
    assert 3.0 < ratio < 5.5, dh
    # links stay in SU(3)
    np.testing.assert_allclose(np.linalg.det(u1), 1.0, atol=1e-12)


def test_trajectory_accept_rule():
    dims, kappa, mu, beta = (2, 2, 2, 2), 0.155, 0.01, 5.0
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, 95)
    p = synth.gaussian_momenta(v, 96)
    eta = synth.gaussian_spinor(v, 97)
    out = H.trajectory(U, p, eta, 0.5, dims, kappa, mu, BC, beta, n_steps=10, dt=0.1)
    assert out["accepted"] == (0.5 < np.exp(-out["dH"]))
    # a uniform draw of 0 always accepts, of 1 accepts only when dH <= 0
    assert H.trajectory(U, p, eta, 0.0, dims, kappa, mu, BC, beta, 10, 0.1)["accepted"]


# The standard su(3) structure constants f^abc (1-based labels, totally antisymmetric):
# the non-zero ones up to permutation.
_F_ABC = {(1, 2, 3): 1.0, (1, 4, 7): 0.5, (1, 5, 6): -0.5, (2, 4, 6): 0.5, (2, 5, 7): 0.5, (3, 4, 5): 0.5,
          (3, 6, 7): -0.5, (4, 5, 8): np.sqrt(3) / 2, (6, 7, 8): np.sqrt(3) / 2}


def test_oracle_su3_generators_are_the_gell_mann_basis():
    """T^a = lambda^a / 2: hermitian, traceless, Tr T^a T^b = delta^ab / 2, and
    [T^a, T^b] = i f^abc T^c with the textbook f^abc (f^123 = 1, f^458 = sqrt(3)/2, ...).
    A swapped label, a sign or a factor in any entry breaks one of these."""
    T = F.T_GEN
    assert T.shape == (8, 3, 3)
    for a in range(8):
        assert np.allclose(T[a], T[a].conj().T, atol=1e-15)
        assert abs(np.trace(T[a])) < 1e-15
    gram = np.einsum("aij,bji->ab", T, T)
    assert np.allclose(gram, 0.5 * np.eye(8), atol=1e-15)
    want = np.zeros((8, 8, 8))
    for (a, b, c), v in _F_ABC.items():
        for (i, j, k), s in (((a, b, c), 1), ((b, c, a), 1), ((c, a, b), 1), ((b, a, c), -1), ((a, c, b), -1),
                             ((c, b, a), -1)):
            want[i - 1, j - 1, k - 1] = s * v
    comm = np.einsum("aij,bjk->abik", T, T) - np.einsum("bij,ajk->abik", T, T)
    # f^abc = -2 i Tr([T^a, T^b] T^c)
    f = (-2j * np.einsum("abik,cki->abc", comm, T)).real
    assert np.allclose(f, want, atol=1e-14)
    assert np.allclose((-2j * np.einsum("abik,cki->abc", comm, T)).imag, 0, atol=1e-14)
