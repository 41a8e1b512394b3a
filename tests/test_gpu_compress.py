"""REC10 and REC8 links on the GPU against the FP64 oracle: packing round trips in every precision, every
operator on the parity cases, multi-RHS point sources through the LDS-staged links, CG (FP64 and
FP16-inner), BiCGStab and the fermion force."""
import numpy as np
import pytest

from gpu_util import BC_AP, BC_TWIST, TOL, Fields, dev, host, oracle_op, rel
from oracle import compress as OC
from oracle import dirac as D
from oracle import force as F
from paper_1209_5942_amd import synth
from paper_1209_5942_amd import tmqcd as T

pytestmark = pytest.mark.gpu

ALL_OPS = [T.DSLASH_EO, T.DSLASH_OE, T.M, T.MDAG, T.MDAGM, T.MHAT, T.MHATDAG, T.MHATDAGMHAT]
CASES = {
    "4x4x4x4": ((4, 4, 4, 4), 0.3, 0.15, 0.01, BC_AP),
    "2x2x2x2": ((2, 2, 2, 2), 0.5, 0.16, 0.005, BC_TWIST),
    "12x6x4x10": ((12, 6, 4, 10), 0.5, 0.162, 0.003, BC_TWIST),
}
# reconstruction divides by |a2|^2 + |a3|^2 (2/3 on average for these links): a few units of the storage rounding
PACK_TOL = {T.F64: 1e-13, T.F32: 1e-6, T.F16: 3e-3}


@pytest.fixture(scope="module", params=list(CASES))
def fields(request):
    dims, eps, kappa, mu, bc = CASES[request.param]
    return Fields(dims, eps, 2000 + len(request.param), kappa, mu, bc)


@pytest.mark.parametrize("prec", [T.F64, T.F32, T.F16])
@pytest.mark.parametrize("recon", [T.RECON10, T.RECON8])
def test_pack_roundtrip(prec, recon):
    f = Fields((6, 4, 2, 4), 0.6, 2101, 0.15, 0.0, BC_AP)
    back = host(T.unpack_gauge(f.prob, T.pack_gauge(f.prob, f.U_dev, prec, recon), prec, recon)).reshape(f.U.shape)
    assert rel(back, f.U) < PACK_TOL[prec], rel(back, f.U)
    if prec == T.F64:
        enc = OC.rec10_encode(f.U) if recon == T.RECON10 else OC.rec8_encode(f.U)
        dec = OC.rec10_decode(enc) if recon == T.RECON10 else OC.rec8_decode(enc)
        assert np.abs(back - dec).max() < 1e-13


@pytest.mark.parametrize("op", ALL_OPS)
@pytest.mark.parametrize("prec", [T.F64, T.F32, T.F16])
@pytest.mark.parametrize("recon", [T.RECON10, T.RECON8])
def test_operator_matches_oracle(fields, op, prec, recon):
    f = fields
    sub_in, sub_out = T.OP_SUBSETS[op]
    psi = f.spinor(sub_in, 78)
    inp = T.pack_spinor(f.prob, dev(psi), prec, sub_in)
    out = T.dslash(f.prob, f.gauge(prec, recon), inp, op, prec, recon)
    got = host(T.unpack_spinor(f.prob, out, prec, sub_out))
    want = oracle_op(op, f.U, psi, f.dims, f.kappa, f.mu, f.bc)
    tol = TOL[prec] * (4 if op in (T.MDAGM, T.MHATDAGMHAT) else 1) * (2 if prec == T.F16 else 1)
    assert rel(got, want) < tol, (op, prec, recon, rel(got, want))


@pytest.mark.parametrize("prec,recon", [(T.F64, T.RECON8), (T.F64, T.RECON10), (T.F32, T.RECON8),
                                        (T.F16, T.RECON10)])
def test_multi_rhs_point_sources(prec, recon):
    f = Fields((4, 4, 2, 6), 0.5, 2201, 0.155, 0.01, BC_TWIST)
    n = f.prob.volume // 2
    nrhs = 6
    psi = np.zeros((nrhs, n, 4, 3), dtype=np.complex128)
    for k in range(nrhs):
        psi[k, (7 * k) % n, k % 4, k % 3] = 1.0
    inp = T.pack_spinor(f.prob, dev(psi), prec, T.EVEN, nrhs=nrhs)
    out = host(T.unpack_spinor(f.prob, T.dslash(f.prob, f.gauge(prec, recon), inp, T.DSLASH_OE, prec, recon,
                                                nrhs=nrhs), prec, T.ODD, nrhs))
    for k in range(nrhs):
        want = oracle_op(T.DSLASH_OE, f.U, psi[k], f.dims, f.kappa, f.mu, f.bc)
        assert rel(out[k], want) < TOL[prec] * 2, (k, rel(out[k], want))


@pytest.mark.parametrize("inner", [T.F64, T.F16])
def test_cg_with_rec8_links(inner):
    f = Fields((8, 4, 4, 8), 0.4, 2301, 0.16, 0.01, BC_AP)
    b = f.spinor(T.EVEN, 2302)
    gauges = {T.F64: f.gauge(T.F64, T.RECON8), inner: f.gauge(inner, T.RECON8)}
    x, st, rc = T.cg(f.prob, gauges, T.pack_spinor(f.prob, dev(b), T.F64, T.EVEN), tol=1e-10, op=T.MHATDAGMHAT,
                     inner_prec=inner, recon=T.RECON8)
    assert rc == T.OK
    # The solver's system is the one on the reconstructed links, which differ from U by the
    # FP64 rounding of the stored numbers times the reconstruction's 1/(|a2|^2 + |a3|^2) (up to
    # 1e-13 here): the oracle rebuilds the same links from its own encoding and checks the
    # requested 1e-10 on them; the two reconstructions differ by a few ulp, which moves the
    # residual by cond(A) times that, far below the 2 % allowed on top.
    Ur = OC.rec8_decode(OC.rec8_encode(f.U))
    A = lambda v: D.apply_MhatdagMhat(Ur, v, f.dims, f.kappa, f.mu, f.bc)
    assert D.true_rel_residual(A, b, host(T.unpack_spinor(f.prob, x, T.F64, T.EVEN))) <= 1.02e-10


def test_bicgstab_with_rec10_links():
    f = Fields((8, 4, 4, 8), 0.4, 2401, 0.16, 0.01, BC_TWIST)
    b = f.spinor(T.FULL, 2402)
    x, st, rc = T.bicgstab(f.prob, f.gauge(T.F64, T.RECON10), T.pack_spinor(f.prob, dev(b)), tol=1e-10, op=T.M,
                           recon=T.RECON10)
    assert rc == T.OK
    # as for CG above: the residual of the system on the reconstructed links
    Ur = OC.rec10_decode(OC.rec10_encode(f.U))
    A = lambda v: D.apply_M(Ur, v, f.dims, f.kappa, f.mu, f.bc)
    assert D.true_rel_residual(A, b, host(T.unpack_spinor(f.prob, x))) <= 1.02e-10


@pytest.mark.parametrize("recon", [T.RECON10, T.RECON8])
def test_force_with_compressed_links(recon):
    f = Fields((4, 4, 2, 4), 0.5, 2501, 0.155, 0.01, BC_TWIST)
    x = synth.gaussian_spinor(f.prob.volume, 2502)
    y = synth.gaussian_spinor(f.prob.volume, 2503)
    got = host(T.force(f.prob, f.gauge(T.F64, recon), T.pack_spinor(f.prob, dev(x)), T.pack_spinor(f.prob, dev(y)),
                       recon=recon))
    assert rel(got, F.fermion_force(f.U, x, y, f.dims, f.kappa, f.bc)) < 1e-12
