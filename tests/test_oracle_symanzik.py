"""Pins for the oracle's tree-level Symanzik gauge action and its force (no GPU).

* The unit field has zero action and Re Tr R = 3 on all 12 V rectangles.
* A weak abelian plane wave U_x(y) = diag(e^{iA}, e^{-iA}, 1), A = eps sin(k y),
  all other links 1: the action equals its closed form
      (beta/3) V_perp (L_y/2) eps^2 [c0 4 sin^2(k/2) + c1 (16 sin^2(k/2) + 4 sin^2 k)]
  (pins the rectangle shapes, both orientations and the counting), and its
  lattice artefact relative to the continuum value falls as k^2 at c1 = 0 but
  as k^4 at c1 = -1/12, the tree-level improvement that fixes the sign reading.
* Gauge invariance of the action and of the per-link force norm.
* Central finite differences of the action along all eight generators.
* At c1 = 0 the path-walking oracle reproduces the plaquette formulas of force.py.
"""
import numpy as np
import pytest

from oracle import dirac as D
from oracle import force as F
from oracle import hmc as H
from oracle import symanzik as S
from paper_1209_5942_amd import synth

C1 = -1.0 / 12.0


def _plane_wave(dims, eps, n):
    """The abelian plane wave along y (links in canonical (V, 4, 3, 3) layout) and its wave number."""
    v = int(np.prod(dims))
    k = 2.0 * np.pi * n / dims[1]
    y = D.coords(dims)[:, 1]
    a = eps * np.sin(k * y)
    U = np.tile(np.eye(3, dtype=np.complex128), (v, 4, 1, 1))
    U[:, 0, 0, 0] = np.exp(1j * a)
    U[:, 0, 1, 1] = np.exp(-1j * a)
    return U, k


def test_unit_field():
    dims = (2, 4, 2, 4)
    v = int(np.prod(dims))
    U = np.tile(np.eye(3, dtype=np.complex128), (v, 4, 1, 1))
    assert S.rectangle_sum(U, dims) == pytest.approx(36.0 * v, abs=1e-12)
    assert abs(S.action(U, dims, 5.0, C1)) < 1e-12
    assert np.abs(S.force(U, dims, 5.0, C1)).max() < 1e-14


@pytest.mark.parametrize("c1", [0.0, C1, 0.3])
def test_abelian_plane_wave_closed_form(c1):
    dims, eps, beta = (2, 16, 2, 2), 1e-3, 6.0
    U, k = _plane_wave(dims, eps, 3)
    c0 = 1.0 - 8.0 * c1
    v_perp = dims[0] * dims[2] * dims[3]
    want = beta / 3.0 * v_perp * dims[1] / 2.0 * eps ** 2 * (
        c0 * 4.0 * np.sin(k / 2) ** 2 + c1 * (16.0 * np.sin(k / 2) ** 2 + 4.0 * np.sin(k) ** 2))
    got = S.action(U, dims, beta, c1)
    assert abs(got / want - 1.0) < 1e-6, (got, want)


def test_tree_level_improvement_fixes_the_sign_of_c1():
    dims, eps, beta = (2, 32, 2, 2), 5e-3, 6.0   # round-off and the eps^2 nonlinearity stay far below k^4/90
    v_perp = dims[0] * dims[2] * dims[3]

    def artefact(c1, n):
        U, k = _plane_wave(dims, eps, n)
        cont = beta / 3.0 * v_perp * dims[1] / 2.0 * eps ** 2 * k ** 2
        return S.action(U, dims, beta, c1) / cont - 1.0
    wilson = artefact(0.0, 2) / artefact(0.0, 1)
    improved = artefact(C1, 2) / artefact(C1, 1)
    assert 3.8 < wilson < 4.2, wilson          # O(k^2): the Wilson action's a^2 artefact
    assert 15.0 < improved < 17.0, improved    # O(k^4): c1 = -1/12 removes it
    assert abs(artefact(C1, 1)) < abs(artefact(0.0, 1)) / 50


def test_gauge_invariance():
    dims, beta = (4, 2, 4, 2), 5.0
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.5, 31)
    om = synth.random_gauge_transform(v, 2.0, 32)
    c = D.coords(dims)
    ug = np.empty_like(U)
    for m in range(4):
        cf = c.copy()
        cf[:, m] = (cf[:, m] + 1) % dims[m]
        fwd = cf[:, 0] + dims[0] * (cf[:, 1] + dims[1] * (cf[:, 2] + dims[2] * cf[:, 3]))
        ug[:, m] = om @ U[:, m] @ om[fwd].conj().transpose(0, 2, 1)
    s0 = S.action(U, dims, beta, C1)
    assert abs(S.action(ug, dims, beta, C1) - s0) < 1e-11 * abs(s0)
    n0 = np.sum(S.force(U, dims, beta, C1) ** 2, axis=-1)
    n1 = np.sum(S.force(ug, dims, beta, C1) ** 2, axis=-1)
    np.testing.assert_allclose(n1, n0, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("c1", [C1, 0.2])
def test_force_vs_finite_differences(c1):
    dims, beta = (4, 2, 2, 4), 5.0
    U = synth.random_links(dims, 0.5, 41)
    G = S.force(U, dims, beta, c1)
    h = 1e-5
    for site, m in [(0, 0), (5, 1), (17, 2), (63, 3), (2, 3), (9, 0)]:
        for a in range(8):
            up, um = U.copy(), U.copy()
            up[site, m] = H.su3_exp(h * np.eye(8)[a], 1.0) @ U[site, m]
            um[site, m] = H.su3_exp(-h * np.eye(8)[a], 1.0) @ U[site, m]
            fd = (S.action(up, dims, beta, c1) - S.action(um, dims, beta, c1)) / (2 * h)
            assert abs(fd - G[site, m, a]) < 1e-7 * max(1.0, np.abs(G).max()), (site, m, a, fd, G[site, m, a])


def test_plaquette_part_matches_force_module():
    dims, beta = (4, 2, 2, 4), 5.0
    U = synth.random_links(dims, 0.5, 51)
    assert abs(S.plaquette_sum(U, dims) - F.plaquette_sum(U, dims)) < 1e-11
    assert abs(S.action(U, dims, beta, 0.0) - F.gauge_action(U, dims, beta)) < 1e-10
    assert np.abs(S.force(U, dims, beta, 0.0) - F.gauge_force(U, dims, beta)).max() < 1e-12
