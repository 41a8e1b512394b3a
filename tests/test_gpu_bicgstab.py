"""BiCGStab on M and on the even-odd Schur complement Mhat, through the C ABI, against the FP64 oracle:
the oracle recomputes ||b - A x|| / ||b|| of the returned solution, dense LU on 2^4, the solution of the
oracle's own BiCGStab, a nonzero start, b = 0, the iteration cap, REC12 links, and a 24^3 x 48 solve."""
import numpy as np
import pytest

from gpu_util import BC_AP, BC_TWIST, Fields, cached_fields, dev, host
from oracle import bicgstab as OB
from oracle import dirac as D
from paper_1209_5942_amd import synth
from paper_1209_5942_amd import tmqcd as T

pytestmark = pytest.mark.gpu


def _op_fns(f, op):
    if op == T.M:
        return T.FULL, (lambda v: D.apply_M(f.U, v, f.dims, f.kappa, f.mu, f.bc)), f.prob.volume
    return T.EVEN, (lambda v: D.apply_Mhat(f.U, v, f.dims, f.kappa, f.mu, f.bc)), f.prob.volume // 2


@pytest.mark.parametrize("op", [T.M, T.MHAT])
@pytest.mark.parametrize("dims,bc,recon", [((4, 4, 4, 4), BC_AP, T.RECON18), ((12, 6, 4, 10), BC_TWIST, T.RECON18),
                                           ((4, 2, 6, 4), BC_TWIST, T.RECON12)])
def test_bicgstab_residual_by_oracle(op, dims, bc, recon):
    print(f"\nbicgstab op={op} dims={dims} recon={recon}", flush=True)
    f = Fields(dims, 0.4, 501, 0.16, 0.01, bc)
    subset, A, n = _op_fns(f, op)
    b = synth.gaussian_spinor(n, 502)
    bd = T.pack_spinor(f.prob, dev(b), T.F64, subset)
    x, st, rc = T.bicgstab(f.prob, f.gauge(T.F64, recon), bd, tol=1e-10, op=op, recon=recon)
    assert rc == T.OK and st["converged"] == 1
    xs = host(T.unpack_spinor(f.prob, x, T.F64, subset))
    res = D.true_rel_residual(A, b, xs)
    assert res <= 1e-10, res
    assert abs(st["true_rel_residual"] - res) < 1e-3 * res + 1e-14
    # the oracle's BiCGStab reaches the same solution within the tolerance's reach
    xo, _, ok = OB.bicgstab(A, b, 1e-12)
    assert ok and np.linalg.norm(xs - xo) / np.linalg.norm(xo) < 1e-8


@pytest.mark.parametrize("op", [T.M, T.MHAT])
def test_bicgstab_against_dense_lu_2x2x2x2(op):
    f = Fields((2, 2, 2, 2), 0.5, 511, 0.15, 0.05, BC_TWIST)
    subset, A, n = _op_fns(f, op)
    b = synth.gaussian_spinor(n, 512)
    x, st, rc = T.bicgstab(f.prob, f.gauge(T.F64, 0), T.pack_spinor(f.prob, dev(b), T.F64, subset), tol=1e-12,
                           op=op)
    xs = host(T.unpack_spinor(f.prob, x, T.F64, subset))
    want = np.linalg.solve(D.dense_matrix(A, n), b.reshape(-1)).reshape(b.shape)
    assert np.linalg.norm(xs - want) / np.linalg.norm(want) < 1e-10


def test_bicgstab_nonzero_start_zero_source_and_cap():
    f = Fields((4, 4, 4, 4), 0.4, 521, 0.16, 0.01, BC_AP)
    subset, A, n = _op_fns(f, T.MHAT)
    g = f.gauge(T.F64, 0)
    b = synth.gaussian_spinor(n, 522)
    bd = T.pack_spinor(f.prob, dev(b), T.F64, subset)
    x, st, _ = T.bicgstab(f.prob, g, bd, tol=1e-12, op=T.MHAT)
    # from the converged solution: no iteration
    x2 = x.clone()
    _, st2, rc2 = T.bicgstab(f.prob, g, bd, x2, x_is_zero=False, tol=1e-10, op=T.MHAT)
    assert rc2 == T.OK and st2["iters"] == 0
    # from a perturbed start: converges, residual by the oracle
    x3 = T.pack_spinor(f.prob, dev(host(T.unpack_spinor(f.prob, x, T.F64, subset)) + 0.1 * synth.gaussian_spinor(n, 523)),
                       T.F64, subset)
    _, st3, rc3 = T.bicgstab(f.prob, g, bd, x3, x_is_zero=False, tol=1e-10, op=T.MHAT)
    assert rc3 == T.OK
    assert D.true_rel_residual(A, b, host(T.unpack_spinor(f.prob, x3, T.F64, subset))) <= 1e-10
    # b = 0 gives x = 0 at once
    z = T.pack_spinor(f.prob, dev(np.zeros((n, 4, 3), dtype=np.complex128)), T.F64, subset)
    xz, stz, rcz = T.bicgstab(f.prob, g, z, tol=1e-10, op=T.MHAT)
    assert rcz == T.OK and stz["iters"] == 0 and not host(T.unpack_spinor(f.prob, xz, T.F64, subset)).any()
    # the iteration cap
    _, stc, rcc = T.bicgstab(f.prob, g, bd, tol=1e-14, op=T.MHAT, max_iter=3, raise_on_noconv=False)
    assert rcc == T.ENOCONV and stc["iters"] == 3 and stc["converged"] == 0


@pytest.mark.timeout(300)
def test_bicgstab_24x24x24x48_by_oracle():
    dims = (24, 24, 24, 48)
    print(f"\nbicgstab {dims}", flush=True)
    f = cached_fields(dims, 0.5, 17, 0.16, 0.005)
    subset, A, n = _op_fns(f, T.MHAT)
    b = synth.gaussian_spinor(n, 531)
    x, st, rc = T.bicgstab(f.prob, f.gauge(T.F64, 0), T.pack_spinor(f.prob, dev(b), T.F64, subset), tol=1e-10,
                           op=T.MHAT)
    assert rc == T.OK
    res = D.true_rel_residual(A, b, host(T.unpack_spinor(f.prob, x, T.F64, subset)))
    print(f"iters {st['iters']}, oracle residual {res:.2e}", flush=True)
    assert res <= 1e-10
