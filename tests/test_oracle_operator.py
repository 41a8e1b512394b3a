"""Pins for the FP64 oracle of the twisted-mass operator (no GPU).

Nothing in the paper prints an operator value, so every pin is a closed form,
an invariant or an independent brute-force construction:

* free-field (U = 1) momentum-space spectra of M, M^dag M and the Schur
  complement Mhat (closed forms derived from the operator's definition);
* gamma5-hermiticity, the twisted-mass shift identity behind the paper's
  two-flavour determinant statement, and gauge covariance;
* the matrix built block by block from its matrix elements (the paper's
  delta_{x+mu,y} form), densely on 2^4 and sparsely on a 2x4x6x8 lattice whose
  four extents differ, so that a swapped axis cannot pass;
* the Schur complement built densely from the blocks of M, the even-odd solve
  and CG against dense LU.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dirac as D
from paper_1209_5942_amd import synth

BC_AP = (1, 1, 1, -1)

# The documented chiral basis, written out entry by entry (independent of the oracle's
# construction from Pauli matrices): gamma_x, gamma_y, gamma_z, gamma_t and gamma5.
_i = 1j
GAMMA_REF = np.array([
    [[0, 0, 0, -_i], [0, 0, -_i, 0], [0, _i, 0, 0], [_i, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, -_i, 0], [0, 0, 0, _i], [_i, 0, 0, 0], [0, -_i, 0, 0]],
    [[0, 0, -1, 0], [0, 0, 0, -1], [-1, 0, 0, 0], [0, -1, 0, 0]],
], dtype=np.complex128)
GAMMA5_REF = np.diag([-1, -1, 1, 1]).astype(np.complex128)
BC_TWIST = (np.exp(0.3j), np.exp(0.7j), -1.0, np.exp(1.1j))


def _momenta(dims):
    """Allowed momenta: periodic in space, antiperiodic in time; shape (V, 4)."""
    lx, ly, lz, lt = dims
    ax = [2 * np.pi * np.arange(lx) / lx, 2 * np.pi * np.arange(ly) / ly,
          2 * np.pi * np.arange(lz) / lz, (2 * np.arange(lt) + 1) * np.pi / lt]
    grid = np.meshgrid(*ax, indexing="ij")
    return np.stack([g.reshape(-1) for g in grid], axis=1)


def _free_spectrum_M(dims, kappa, mu):
    # M(p) = a + i B, a = 1 - 2 kappa sum cos p, B hermitian with
    # B^2 = 4 kappa^2 (sum sin^2 p + mu^2); each sign six-fold (2 spins x 3 colours)
    p = _momenta(dims)
    a = 1 - 2 * kappa * np.cos(p).sum(1)
    b = 2 * kappa * np.sqrt((np.sin(p) ** 2).sum(1) + mu ** 2)
    return np.repeat(np.concatenate([a + 1j * b, a - 1j * b]), 6)


def _free_spectrum_Mhat(dims, kappa, mu):
    # even-site Schur complement: alpha +- i sqrt(beta1^2 s^2 + beta2^2); the
    # momenta p and p + (pi,pi,pi,pi) give the same value, three-fold each
    p = _momenta(dims)
    w = 2 * kappa * mu
    c = np.cos(p).sum(1)
    s2 = (np.sin(p) ** 2).sum(1)
    alpha = 1 - 4 * kappa ** 2 * (c ** 2 - s2) / (1 + w ** 2)
    beta1 = 8 * kappa ** 2 * c / (1 + w ** 2)
    beta2 = w + 4 * w * kappa ** 2 * (c ** 2 + s2) / (1 + w ** 2)
    r = np.sqrt(beta1 ** 2 * s2 + beta2 ** 2)
    return np.repeat(np.concatenate([alpha + 1j * r, alpha - 1j * r]), 3)


def _assert_same_multiset(got, want, tol=1e-10):
    assert got.shape == want.shape
    np.testing.assert_allclose(np.sort(got.real), np.sort(want.real), atol=tol)
    np.testing.assert_allclose(np.sort(got.imag), np.sort(want.imag), atol=tol)
    for z0 in (0.37 + 0.81j, -1.3 + 0.2j):
        np.testing.assert_allclose(np.sort(np.abs(got - z0)), np.sort(np.abs(want - z0)), atol=tol)


def _dense(op, dims, kappa, mu, bc, U, n_sites=None):
    n = int(np.prod(dims)) if n_sites is None else n_sites
    return D.dense_matrix(lambda v: op(U, v, dims, kappa, mu, bc), n)


def _block_matrix(U, dims, kappa, mu, bc, sparse=False):
    """M assembled from its matrix elements: diagonal (1 + i w gamma5) (x) 1_c, and for
    every link x -> y = x + mu the blocks -kappa b (1 - gamma_mu) (x) U_mu(x) at (x, y)
    and -kappa conj(b) (1 + gamma_mu) (x) U_mu(x)^dag at (y, x).  Blocks add, so on an
    extent-2 direction both neighbours of a site land on the same block."""
    lx, ly, lz, lt = dims
    v = lx * ly * lz * lt
    ext = (lx, ly, lz, lt)
    rows, cols, vals = [], [], []

    def add(i, j, blk):
        r, c = np.nonzero(np.ones((12, 12)))
        rows.append(12 * i + r)
        cols.append(12 * j + c)
        vals.append(blk.reshape(-1))

    a = np.kron(np.eye(4) + 2j * kappa * mu * GAMMA5_REF, np.eye(3))
    for s in range(v):
        add(s, s, a)
        c = [s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)]
        for m in range(4):
            cf = list(c)
            cf[m] = (c[m] + 1) % ext[m]
            y = cf[0] + lx * (cf[1] + ly * (cf[2] + lz * cf[3]))
            b = complex(bc[m]) if c[m] == ext[m] - 1 else 1.0
            add(s, y, -kappa * b * np.kron(np.eye(4) - GAMMA_REF[m], U[s, m]))
            add(y, s, -kappa * np.conj(b) * np.kron(np.eye(4) + GAMMA_REF[m], U[s, m].conj().T))
    mat = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                        shape=(12 * v, 12 * v)).tocsr()   # duplicates are summed
    return mat if sparse else mat.toarray()


def test_gamma_basis():
    np.testing.assert_array_equal(D.GAMMA, GAMMA_REF)
    for m in range(4):
        assert np.allclose(D.GAMMA[m], D.GAMMA[m].conj().T)
        for n in range(4):
            ac = D.GAMMA[m] @ D.GAMMA[n] + D.GAMMA[n] @ D.GAMMA[m]
            assert np.allclose(ac, 2 * np.eye(4) * (m == n))
    assert np.allclose(D.GAMMA5, np.diag([-1, -1, 1, 1]))


@pytest.mark.parametrize("kappa", [0.15, 0.162])
@pytest.mark.parametrize("mu", [0.0, 0.01])
def test_free_field_spectrum_M_2x2x2x2(kappa, mu):
    dims = (2, 2, 2, 2)
    m = _dense(D.apply_M, dims, kappa, mu, BC_AP, synth.unit_links(dims))
    _assert_same_multiset(np.linalg.eigvals(m), _free_spectrum_M(dims, kappa, mu))


def test_free_field_spectrum_M_4x2x2x4():
    dims, kappa, mu = (4, 2, 2, 4), 0.162, 0.003
    m = _dense(D.apply_M, dims, kappa, mu, BC_AP, synth.unit_links(dims))
    _assert_same_multiset(np.linalg.eigvals(m), _free_spectrum_M(dims, kappa, mu))


def test_free_field_massless_at_kappa_one_eighth():
    # kappa = 1/(2(am + 4)) at am = 0: with periodic time the zero-momentum mode of the
    # free Wilson operator is an exact zero mode (this fixes the hopping prefactor as kappa)
    dims = (2, 2, 2, 2)
    m = _dense(D.apply_M, dims, 0.125, 0.0, (1, 1, 1, 1), synth.unit_links(dims))
    ev = np.linalg.eigvals(m)
    assert np.sum(np.abs(ev) < 1e-12) == 12


@pytest.mark.slow
def test_free_field_spectrum_MdagM_4x4x4x4():
    dims, kappa, mu = (4, 4, 4, 4), 0.15, 0.01
    m = _dense(D.apply_M, dims, kappa, mu, BC_AP, synth.unit_links(dims))
    p = _momenta(dims)
    want = (1 - 2 * kappa * np.cos(p).sum(1)) ** 2 + 4 * kappa ** 2 * ((np.sin(p) ** 2).sum(1) + mu ** 2)
    got = np.linalg.eigvalsh(m.conj().T @ m)
    np.testing.assert_allclose(np.sort(got), np.sort(np.repeat(want, 12)), atol=1e-11)


@pytest.mark.parametrize("dims,kappa,mu", [((4, 2, 2, 4), 0.15, 0.01), ((4, 4, 4, 4), 0.162, 0.003)])
def test_free_field_spectrum_Mhat(dims, kappa, mu):
    n_even = int(np.prod(dims)) // 2
    m = _dense(D.apply_Mhat, dims, kappa, mu, BC_AP, synth.unit_links(dims), n_even)
    _assert_same_multiset(np.linalg.eigvals(m), _free_spectrum_Mhat(dims, kappa, mu))


def test_dense_block_matrix_2x2x2x2():
    dims, kappa, mu = (2, 2, 2, 2), 0.15, 0.01
    U = synth.random_links(dims, 0.3, 7)
    want = _block_matrix(U, dims, kappa, mu, BC_TWIST)
    np.testing.assert_allclose(_dense(D.apply_M, dims, kappa, mu, BC_TWIST, U), want, atol=1e-14)
    np.testing.assert_allclose(_dense(D.apply_Mdag, dims, kappa, mu, BC_TWIST, U), want.conj().T,
                               atol=1e-14)


def test_sparse_block_matrix_distinct_extents():
    dims, kappa, mu = (2, 4, 6, 8), 0.16, 0.005
    U = synth.random_links(dims, 0.5, 8)
    v = int(np.prod(dims))
    mat = _block_matrix(U, dims, kappa, mu, BC_TWIST, sparse=True)
    psi = synth.gaussian_spinor(v, 9)
    np.testing.assert_allclose(D.apply_M(U, psi, dims, kappa, mu, BC_TWIST).reshape(-1),
                               mat @ psi.reshape(-1), atol=1e-13)
    np.testing.assert_allclose(D.apply_Mdag(U, psi, dims, kappa, mu, BC_TWIST).reshape(-1),
                               mat.conj().T @ psi.reshape(-1), atol=1e-13)


def test_hop_at_sites_matches_whole_lattice():
    dims = (2, 4, 6, 8)
    U = synth.random_links(dims, 0.5, 3)
    psi = synth.gaussian_spinor(int(np.prod(dims)), 4)
    full = D.hop(U, psi, dims, BC_TWIST)
    sites = np.arange(0, int(np.prod(dims)), 7)
    np.testing.assert_allclose(D.hop_at_sites(U, psi, dims, BC_TWIST, sites), full[sites], atol=1e-13)


def test_gamma5_hermiticity_random_field():
    dims, kappa, mu = (4, 4, 4, 4), 0.15, 0.01
    U = synth.random_links(dims, 0.3, 1)
    v = int(np.prod(dims))
    chi, psi = synth.gaussian_spinor(v, 2), synth.gaussian_spinor(v, 3)
    lhs = np.vdot(chi, D.apply_M(U, psi, dims, kappa, mu, BC_TWIST))
    g5m = D.gamma5(D.apply_M(U, D.gamma5(chi), dims, kappa, -mu, BC_TWIST))
    assert abs(lhs - np.vdot(g5m, psi)) < 1e-12 * abs(lhs)
    # the same for the Schur complement on even sites
    ce, pe = D.to_half(chi, dims, 0), D.to_half(psi, dims, 0)
    lhs = np.vdot(ce, D.apply_Mhat(U, pe, dims, kappa, mu, BC_TWIST))
    g5m = D.gamma5(D.apply_Mhat(U, D.gamma5(ce), dims, kappa, -mu, BC_TWIST))
    assert abs(lhs - np.vdot(g5m, pe)) < 1e-12 * abs(lhs)
    # and Mhat^dag as implemented is the adjoint of Mhat
    rhs = np.vdot(D.apply_Mhatdag(U, ce, dims, kappa, mu, BC_TWIST), pe)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_twisted_mass_shift_identity():
    # M(mu)^dag M(mu) = M(0)^dag M(0) + 4 kappa^2 mu^2: the two-flavour determinant statement
    dims, kappa, mu = (4, 4, 4, 4), 0.16, 0.05
    U = synth.random_links(dims, 0.5, 11)
    psi = synth.gaussian_spinor(int(np.prod(dims)), 12)
    a = D.apply_MdagM(U, psi, dims, kappa, mu, BC_AP)
    b = D.apply_MdagM(U, psi, dims, kappa, 0.0, BC_AP) + 4 * kappa ** 2 * mu ** 2 * psi
    np.testing.assert_allclose(a, b, atol=1e-13)


def test_gauge_covariance():
    dims, kappa, mu = (4, 4, 2, 6), 0.15, 0.01
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, 21)
    om = synth.random_gauge_transform(v, 2.0, 22)
    psi = synth.gaussian_spinor(v, 23)
    fwd = np.empty(v, dtype=np.int64)
    ug = np.empty_like(U)
    c = D.coords(dims)
    for m in range(4):
        cf = c.copy()
        cf[:, m] = (cf[:, m] + 1) % dims[m]
        fwd = cf[:, 0] + dims[0] * (cf[:, 1] + dims[1] * (cf[:, 2] + dims[2] * cf[:, 3]))
        ug[:, m] = om @ U[:, m] @ om[fwd].conj().transpose(0, 2, 1)
    rot = lambda f: np.einsum("nab,nsb->nsa", om, f)
    lhs = D.apply_M(ug, rot(psi), dims, kappa, mu, BC_TWIST)
    rhs = rot(D.apply_M(U, psi, dims, kappa, mu, BC_TWIST))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)
    n1 = np.linalg.norm(D.apply_M(U, psi, dims, kappa, mu, BC_TWIST))
    assert abs(np.linalg.norm(lhs) - n1) < 1e-13 * n1


def test_schur_complement_from_blocks_and_eo_solve():
    dims, kappa, mu = (4, 2, 2, 4), 0.15, 0.01
    U = synth.random_links(dims, 0.3, 31)
    m = _block_matrix(U, dims, kappa, mu, BC_TWIST)
    idx = lambda s: (12 * s[:, None] + np.arange(12)[None, :]).reshape(-1)
    e, o = idx(D.half_sites(dims, 0)), idx(D.half_sites(dims, 1))
    schur = m[np.ix_(e, e)] - m[np.ix_(e, o)] @ np.linalg.solve(m[np.ix_(o, o)], m[np.ix_(o, e)])
    n_even = int(np.prod(dims)) // 2
    got = _dense(D.apply_Mhat, dims, kappa, mu, BC_TWIST, U, n_even)
    np.testing.assert_allclose(got, schur, atol=1e-13)
    got_dag = _dense(D.apply_Mhatdag, dims, kappa, mu, BC_TWIST, U, n_even)
    np.testing.assert_allclose(got_dag, schur.conj().T, atol=1e-13)
    b = synth.gaussian_spinor(int(np.prod(dims)), 32)
    x = D.solve_eo(U, b, dims, kappa, mu, BC_TWIST)
    x_lu = np.linalg.solve(m, b.reshape(-1)).reshape(b.shape)
    assert np.linalg.norm(x - x_lu) < 1e-11 * np.linalg.norm(x_lu)


def test_cg_matches_dense_solve():
    dims, kappa, mu = (4, 2, 2, 4), 0.15, 0.0
    U = synth.random_links(dims, 0.3, 41)
    m = _block_matrix(U, dims, kappa, mu, BC_AP)
    b = synth.gaussian_spinor(int(np.prod(dims)), 42)
    x, iters = D.cg(lambda v: D.apply_MdagM(U, v, dims, kappa, mu, BC_AP), b, 1e-12)
    x_lu = np.linalg.solve(m.conj().T @ m, b.reshape(-1))
    assert iters > 10
    assert np.linalg.norm(x.reshape(-1) - x_lu) < 1e-10 * np.linalg.norm(x_lu)
    # (M^dag M)^{-1} = M^{-1} M^{-dag}
    x2 = np.linalg.solve(m, np.linalg.solve(m.conj().T, b.reshape(-1)))
    assert np.linalg.norm(x2 - x_lu) < 1e-12 * np.linalg.norm(x_lu)


def test_links_are_special_unitary_and_rec12_rebuilds_third_row():
    # 12-real storage keeps rows 1 and 2; row 3 = conj(row1 x row2) when det U = 1
    U = synth.random_links((4, 4, 2, 2), 0.5, 5).reshape(-1, 3, 3)
    np.testing.assert_allclose(U @ U.conj().transpose(0, 2, 1), np.broadcast_to(np.eye(3), U.shape),
                               atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(U), 1.0, atol=1e-14)
    np.testing.assert_allclose(np.conj(np.cross(U[:, 0], U[:, 1])), U[:, 2], atol=1e-14)
