"""Pins for the oracle's BiCGStab (no GPU): its solutions of M x = b and Mhat x_e = b_e against dense LU,
the true residual, b = 0, a start from the solution, and a non-hermitian textbook system."""
import numpy as np
import pytest

from oracle import bicgstab as B
from oracle import dirac as D
from paper_1209_5942_amd import synth

BC = (np.exp(0.3j), 1.0, np.exp(-0.4j), -1.0)


def test_small_nonsymmetric_matrix_against_lu():
    rng = np.random.default_rng(5)
    n = 40
    a = np.eye(n) * 4 + rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) * 0.5
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    x, k, ok = B.bicgstab(lambda v: a @ v, b, 1e-13)
    assert ok
    np.testing.assert_allclose(x, np.linalg.solve(a, b), rtol=0, atol=1e-11 * np.abs(np.linalg.solve(a, b)).max())


@pytest.mark.parametrize("dims,kappa,mu", [((2, 2, 2, 2), 0.15, 0.01), ((4, 2, 2, 4), 0.16, 0.3)])
def test_M_against_dense_lu(dims, kappa, mu):
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, 61)
    b = synth.gaussian_spinor(v, 62)
    A = lambda f: D.apply_M(U, f, dims, kappa, mu, BC)
    x, k, ok = B.bicgstab(A, b, 1e-12)
    assert ok
    assert D.true_rel_residual(A, b, x) < 2e-12
    m = D.dense_matrix(A, v)
    want = np.linalg.solve(m, b.reshape(-1)).reshape(b.shape)
    assert np.linalg.norm(x - want) / np.linalg.norm(want) < 1e-10


def test_Mhat_against_dense_lu_and_the_full_solve():
    dims, kappa, mu = (4, 2, 2, 4), 0.16, 0.02
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, 63)
    be = synth.gaussian_spinor(v // 2, 64)
    A = lambda f: D.apply_Mhat(U, f, dims, kappa, mu, BC)
    x, k, ok = B.bicgstab(A, be, 1e-12)
    assert ok
    m = D.dense_matrix(A, v // 2)
    want = np.linalg.solve(m, be.reshape(-1)).reshape(be.shape)
    assert np.linalg.norm(x - want) / np.linalg.norm(want) < 1e-10
    # the even half of the full solution of M x = (b_e, 0) solves the same Schur system
    # up to the factor of the asymmetric complement: Mhat x_e = b_e - kappa H_eo A^-1 0 = b_e
    full_b = D.to_full(be, dims, 0)
    xf, _, _ = B.bicgstab(lambda f: D.apply_M(U, f, dims, kappa, mu, BC), full_b, 1e-13)
    xe = xf[D.half_sites(dims, 0)]
    assert np.linalg.norm(xe - want) / np.linalg.norm(want) < 1e-10


def test_zero_source_and_exact_start():
    dims, kappa, mu = (2, 2, 2, 2), 0.15, 0.01
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.4, 65)
    A = lambda f: D.apply_M(U, f, dims, kappa, mu, BC)
    x, k, ok = B.bicgstab(A, np.zeros((v, 4, 3), dtype=np.complex128))
    assert ok and k == 0 and not x.any()
    b = synth.gaussian_spinor(v, 66)
    x1, _, _ = B.bicgstab(A, b, 1e-13)
    x2, k2, ok2 = B.bicgstab(A, b, 1e-10, x0=x1)
    assert ok2 and k2 == 0
