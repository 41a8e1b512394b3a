"""Pins for the plain C++/OpenMP oracle (oracle/cpu/tmqcd_ref.cpp), no GPU.

* every operator against the NumPy oracle (itself pinned by closed forms, dense
  brute force and invariants) on lattices where neighbours coincide (2^4), with
  twisted boundary phases, and on non-cubic extents;
* the free-field closed form: plane waves e^{i p.x} chi are eigenvectors of M^+M
  with eigenvalue (1 - 2 kappa sum cos p)^2 + 4 kappa^2 (sum sin^2 p + mu^2);
* its CG against dense LU on 4^4 and the NumPy oracle's residual;
* results independent of the thread count.
"""
import numpy as np
import pytest

from oracle import cref as R
from oracle import dirac as D
from paper_1209_5942_amd import synth

BC_AP = (1, 1, 1, -1)
BC_TWIST = (np.exp(0.3j), np.exp(0.7j), -1.0, np.exp(1.1j))
CASES = [((4, 4, 4, 4), BC_AP), ((2, 2, 2, 2), BC_TWIST), ((4, 2, 6, 4), BC_TWIST), ((6, 4, 2, 8), BC_AP)]
NUMPY = {"H": lambda U, p, d, k, m, b: D.hop(U, p, d, b), "HOP_EO": lambda U, p, d, k, m, b: D.hop_pq(U, p, d, b, 0),
         "HOP_OE": lambda U, p, d, k, m, b: D.hop_pq(U, p, d, b, 1), "M": D.apply_M, "MDAG": D.apply_Mdag,
         "MDAGM": D.apply_MdagM, "MHAT": D.apply_Mhat, "MHATDAG": D.apply_Mhatdag,
         "MHATDAGMHAT": D.apply_MhatdagMhat}


@pytest.fixture(scope="module", autouse=True)
def _built():
    R.build()


@pytest.mark.parametrize("dims,bc", CASES)
@pytest.mark.parametrize("op", list(NUMPY))
def test_operators_match_numpy_oracle(dims, bc, op):
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.5, 31).reshape(v, 4, 3, 3)
    n = v if op in R.FULL_OPS else v // 2
    psi = synth.gaussian_spinor(n, 32)
    got = R.apply(op, U, psi, dims, 0.16, 0.013, bc)
    want = NUMPY[op](U, psi, dims, 0.16, 0.013, bc)
    assert np.linalg.norm(got - want) <= 1e-14 * np.linalg.norm(want), op


@pytest.mark.parametrize("kappa,mu", [(0.15, 0.01), (0.125, 0.0), (0.162, 0.003)])
def test_free_field_plane_waves_are_eigenvectors(kappa, mu):
    dims = (4, 6, 2, 8)
    v = int(np.prod(dims))
    U = np.tile(np.eye(3, dtype=np.complex128), (v, 4, 1, 1))
    c = D.coords(dims)
    rng = np.random.default_rng(5)
    for n in [(0, 0, 0, 0), (1, 2, 1, 3), (3, 5, 0, 7), (2, 1, 1, 0)]:
        p = np.array([2 * np.pi * n[i] / dims[i] for i in range(3)] + [(2 * n[3] + 1) * np.pi / dims[3]])
        chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
        psi = np.exp(1j * (c @ p))[:, None, None] * chi
        lam = (1 - 2 * kappa * np.cos(p).sum()) ** 2 + 4 * kappa ** 2 * (np.sin(p) ** 2).sum() + 4 * kappa ** 2 * mu ** 2
        out = R.apply("MDAGM", U, psi, dims, kappa, mu, BC_AP)
        assert np.abs(out - lam * psi).max() < 1e-13, n


def test_cg_matches_dense_solve_and_numpy_residual():
    dims, kappa, mu = (4, 4, 4, 4), 0.15, 0.01
    v = 256
    U = synth.random_links(dims, 0.3, 41).reshape(v, 4, 3, 3)
    for op, n in (("MDAGM", v), ("MHATDAGMHAT", v // 2)):
        b = synth.gaussian_spinor(n, 42)
        x, st, rc = R.cg(op, U, b, dims, kappa, mu, BC_AP, tol=1e-12, report_tol=1e-8)
        assert rc == 0 and st["true_rel_residual"] <= 1.1e-12
        A = lambda f: NUMPY[op](U, f, dims, kappa, mu, BC_AP)
        assert D.true_rel_residual(A, b, x) <= 1.1e-12
        assert abs(D.true_rel_residual(A, b, x) - st["true_rel_residual"]) < 1e-14
        assert st["report_iters"] < st["iters"] and st["report_true_rel_residual"] <= 1.1e-8
        dense = D.dense_matrix(lambda f: np.stack([A(g) for g in f]), n)
        xs = np.linalg.solve(dense, b.reshape(-1)).reshape(b.shape)
        assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_thread_count_does_not_change_the_operator():
    dims = (6, 4, 2, 8)
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.5, 51).reshape(v, 4, 3, 3)
    psi = synth.gaussian_spinor(v // 2, 52)
    n0 = R.threads()
    try:
        R.set_threads(1)
        one = R.apply("MHATDAGMHAT", U, psi, dims, 0.16, 0.005, BC_AP)
        R.set_threads(max(2, n0))
        many = R.apply("MHATDAGMHAT", U, psi, dims, 0.16, 0.005, BC_AP)
    finally:
        R.set_threads(n0)
    assert np.array_equal(one, many)


def test_mismatched_sizes_are_rejected_before_the_loops():
    """The C++ loops trust the sizes they are given; the wrapper refuses fields of the wrong size."""
    dims = (4, 4, 4, 4)
    v = int(np.prod(dims))
    U = synth.random_links(dims, 0.5, 41).reshape(v, 4, 3, 3)
    full, half = synth.gaussian_spinor(v, 42), synth.gaussian_spinor(v // 2, 43)
    with pytest.raises(ValueError):
        R.apply("MHAT", U, full, dims, 0.16, 0.01, BC_AP)          # a full field for an even-odd operator
    with pytest.raises(ValueError):
        R.apply("M", U, half, dims, 0.16, 0.01, BC_AP)             # a half field for a full operator
    with pytest.raises(ValueError):
        R.apply("M", U[: v // 2], full, dims, 0.16, 0.01, BC_AP)   # links of another lattice
    with pytest.raises(ValueError):
        R.true_rel_residual("MHATDAGMHAT", U, half, full, dims, 0.16, 0.01, BC_AP)
