"""GPU parity of packing and of every operator of the C interface against the FP64 oracle.

FP64 must match within 1e-12 (relative, global L2), FP32 within 5e-6 and FP16
within 5e-3; a point source has zero sites, so the global norm is the measure.
Sizes: 4^4 (the small configuration), 2^4 (forward and backward neighbours
coincide), a 12x6x4x10 lattice with twisted boundary phases (several workgroups
and a ragged tail), and the 24^3 x 48 production shape checked on sampled sites.
"""
import numpy as np
import pytest

from gpu_util import BC_AP, BC_TWIST, TOL, Fields, cached_fields, dev, host, n_sites, oracle_op, rel
from oracle import dirac as D
from paper_1209_5942_amd import synth
from paper_1209_5942_amd import tmqcd as T

pytestmark = pytest.mark.gpu

ALL_OPS = [T.DSLASH_EO, T.DSLASH_OE, T.M, T.MDAG, T.MDAGM, T.MHAT, T.MHATDAG, T.MHATDAGMHAT]

CASES = {
    "4x4x4x4": ((4, 4, 4, 4), 0.3, 0.15, 0.01, BC_AP),
    "4x4x4x4-mu0": ((4, 4, 4, 4), 0.3, 0.15, 0.0, BC_AP),
    "2x2x2x2": ((2, 2, 2, 2), 0.5, 0.16, 0.005, BC_TWIST),
    "12x6x4x10": ((12, 6, 4, 10), 0.5, 0.162, 0.003, BC_TWIST),
}


@pytest.fixture(scope="module", params=list(CASES))
def fields(request):
    dims, eps, kappa, mu, bc = CASES[request.param]
    return Fields(dims, eps, 1000 + len(request.param), kappa, mu, bc)


@pytest.mark.parametrize("prec", [T.F64, T.F32, T.F16])
@pytest.mark.parametrize("subset", [T.FULL, T.EVEN, T.ODD])
def test_pack_roundtrip(prec, subset):
    prob = T.Problem((6, 4, 2, 4), 0.15, 0.0)
    psi = synth.gaussian_spinor(n_sites(prob, subset), 5, 3)
    psi[1, 7] = 0                                         # an all-zero site (FP16 scale 0)
    packed = T.pack_spinor(prob, dev(psi), prec, subset, nrhs=3)
    back = host(T.unpack_spinor(prob, packed, prec, subset, nrhs=3))
    if prec == T.F64:
        assert np.array_equal(back, psi)
    else:
        assert rel(back, psi) < {T.F32: 1e-7, T.F16: 1e-3}[prec]
        assert np.all(back[1, 7] == 0)


@pytest.mark.parametrize("op", ALL_OPS)
@pytest.mark.parametrize("prec,recon", [(T.F64, T.RECON18), (T.F64, T.RECON12), (T.F32, T.RECON18),
                                        (T.F32, T.RECON12), (T.F16, T.RECON18), (T.F16, T.RECON12)])
def test_operator_matches_oracle(fields, op, prec, recon):
    f = fields
    sub_in, sub_out = T.OP_SUBSETS[op]
    psi = f.spinor(sub_in, 77)
    inp = T.pack_spinor(f.prob, dev(psi), prec, sub_in)
    out = T.dslash(f.prob, f.gauge(prec, recon), inp, op, prec, recon)
    got = host(T.unpack_spinor(f.prob, out, prec, sub_out))
    want = oracle_op(op, f.U, psi, f.dims, f.kappa, f.mu, f.bc)
    tol = TOL[prec] * (4 if op in (T.MDAGM, T.MHATDAGMHAT) else 1)
    assert rel(got, want) < tol, (op, prec, recon, rel(got, want))


@pytest.mark.parametrize("op", [T.DSLASH_OE, T.M, T.MDAG, T.MHATDAGMHAT])
def test_multi_rhs_columns_equal_single_calls(fields, op):
    f = fields
    sub_in, sub_out = T.OP_SUBSETS[op]
    psi = f.spinor(sub_in, 31, nrhs=5)
    inp = T.pack_spinor(f.prob, dev(psi), T.F64, sub_in, nrhs=5)
    out = host(T.unpack_spinor(f.prob, T.dslash(f.prob, f.gauge(T.F64, 0), inp, op, nrhs=5), T.F64, sub_out, 5))
    for k in range(5):
        single = T.dslash(f.prob, f.gauge(T.F64, 0), T.pack_spinor(f.prob, dev(psi[k]), T.F64, sub_in), op)
        one = host(T.unpack_spinor(f.prob, single, T.F64, sub_out))
        assert rel(out[k], one) < 1e-14


@pytest.mark.parametrize("op", ALL_OPS)
@pytest.mark.parametrize("prec,recon", [(T.F64, T.RECON18), (T.F64, T.RECON12), (T.F32, T.RECON12),
                                        (T.F16, T.RECON18)])
def test_multi_rhs_point_sources_match_oracle(fields, op, prec, recon):
    """The 12 spin-colour point sources at site 0 (plus a Gaussian column) through every operator."""
    f = fields
    sub_in, sub_out = T.OP_SUBSETS[op]
    n = n_sites(f.prob, sub_in)
    src = np.concatenate([synth.point_sources(n, 0), f.spinor(sub_in, 41, nrhs=1)], axis=0)   # 13 columns
    inp = T.pack_spinor(f.prob, dev(src), prec, sub_in, nrhs=13)
    out = host(T.unpack_spinor(f.prob, T.dslash(f.prob, f.gauge(prec, recon), inp, op, prec, recon, nrhs=13),
                               prec, sub_out, 13))
    tol = TOL[prec] * (4 if op in (T.MDAGM, T.MHATDAGMHAT) else 1)
    for k in range(13):
        want = oracle_op(op, f.U, src[k], f.dims, f.kappa, f.mu, f.bc)
        assert rel(out[k], want) < tol, (k, rel(out[k], want))


def test_dense_columns_2x2x2x2():
    """M applied to all 192 unit vectors reproduces the oracle's dense matrix."""
    dims, kappa, mu = (2, 2, 2, 2), 0.16, 0.005
    f = Fields(dims, 0.5, 9, kappa, mu, BC_TWIST)
    n = 12 * f.prob.volume
    dense = D.dense_matrix(lambda v: D.apply_M(f.U, v, dims, kappa, mu, BC_TWIST), f.prob.volume)
    got = np.empty((n, n), dtype=np.complex128)
    for j0 in range(0, n, 16):
        e = np.zeros((16, n), dtype=np.complex128)
        e[np.arange(16), np.arange(j0, j0 + 16)] = 1
        inp = T.pack_spinor(f.prob, dev(e.reshape(16, -1, 4, 3)), T.F64, T.FULL, nrhs=16)
        out = T.dslash(f.prob, f.gauge(T.F64, 0), inp, T.M, nrhs=16)
        got[:, j0:j0 + 16] = host(T.unpack_spinor(f.prob, out, T.F64, T.FULL, 16)).reshape(16, n).T
    assert np.abs(got - dense).max() < 1e-14


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec,recon", [(T.F64, T.RECON18), (T.F64, T.RECON12), (T.F32, T.RECON12),
                                        (T.F16, T.RECON12)])
def test_production_shape_sampled(prec, recon):
    """24^3 x 48: whole-lattice hops on the GPU, the oracle on 300 sampled sites."""
    dims, kappa, mu = (24, 24, 24, 48), 0.16, 0.005
    f = cached_fields(dims, 0.5, 24, kappa, mu, BC_AP)
    rng = np.random.default_rng(3)
    psi = synth.gaussian_spinor(f.prob.volume, 25)
    inp = T.pack_spinor(f.prob, dev(psi), prec, T.FULL)
    got = host(T.unpack_spinor(f.prob, T.dslash(f.prob, f.gauge(prec, recon), inp, T.M, prec, recon), prec, T.FULL))
    sites = rng.choice(f.prob.volume, 300, replace=False)
    # boundary sites in every direction are among the samples
    c = D.coords(dims)
    sites = np.unique(np.concatenate([sites, [0, f.prob.volume - 1],
                                      np.nonzero((c[:, 0] == 23) & (c[:, 3] == 47))[0][:8]]))
    want = D.twist(psi[sites], kappa, mu) - kappa * D.hop_at_sites(f.U, psi, dims, BC_AP, sites)
    assert rel(got[sites], want) < TOL[prec]
    # even-odd hop on the same field: the even output of DSLASH_EO is the H_eo part
    ev = D.half_sites(dims, 0)
    inp_o = T.pack_spinor(f.prob, dev(psi[D.half_sites(dims, 1)]), prec, T.ODD)
    got_e = host(T.unpack_spinor(f.prob, T.dslash(f.prob, f.gauge(prec, recon), inp_o, T.DSLASH_EO, prec, recon),
                                 prec, T.EVEN))
    hs = rng.choice(ev.size, 200, replace=False)
    psi_odd_only = psi.copy()
    psi_odd_only[ev] = 0
    want_e = -kappa * D.hop_at_sites(f.U, psi_odd_only, dims, BC_AP, ev[hs])
    assert rel(got_e[hs], want_e) < TOL[prec]


def test_production_shape_gamma5_hermiticity():
    """<chi, Mhat psi> = <Mhat^dag chi, psi> on the whole 24^3 x 48 lattice (holds at any size)."""
    dims = (24, 24, 24, 48)
    f = cached_fields(dims, 0.5, 24, 0.16, 0.005, BC_AP)
    vh = f.prob.volume // 2
    chi, psi = synth.gaussian_spinor(vh, 1), synth.gaussian_spinor(vh, 2)
    g = f.gauge(T.F64, 0)
    mpsi = host(T.unpack_spinor(f.prob, T.dslash(f.prob, g, T.pack_spinor(f.prob, dev(psi), 0, T.EVEN), T.MHAT),
                                0, T.EVEN))
    mdchi = host(T.unpack_spinor(f.prob, T.dslash(f.prob, g, T.pack_spinor(f.prob, dev(chi), 0, T.EVEN),
                                                  T.MHATDAG), 0, T.EVEN))
    a, b = np.vdot(chi, mpsi), np.vdot(mdchi, psi)
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.timeout(600)
def test_production_shape_tuned_launches_sampled():
    """24^3 x 48 in the launch shapes the bench times (tuned single-RHS classes and the tuned 12-RHS
    kernel, FP64 and FP32): the odd<-even hop against the oracle on sampled sites, every column."""
    dims, kappa, mu = (24, 24, 24, 48), 0.16, 0.005
    f = cached_fields(dims, 0.5, 24, kappa, mu, BC_AP)
    rng = np.random.default_rng(11)
    ev, od = D.half_sites(dims, 0), D.half_sites(dims, 1)
    hs = np.unique(np.concatenate([rng.choice(od.size, 120, replace=False), [0, od.size - 1]]))
    try:
        T.tune_clear()
        for prec in (T.F64, T.F32):
            g = f.gauge(prec, T.RECON18)
            T.tune(f.prob, g, prec, T.RECON18)
            T.tune_mrhs(f.prob, g, 12, prec, T.RECON18)
            psi = f.spinor(T.EVEN, 700 + prec, nrhs=12)
            out1 = host(T.unpack_spinor(f.prob, T.dslash(f.prob, g, T.pack_spinor(f.prob, dev(psi[0]), prec, T.EVEN),
                                                         T.DSLASH_OE, prec, T.RECON18), prec, T.ODD))
            outm = host(T.unpack_spinor(f.prob, T.dslash(f.prob, g, T.pack_spinor(f.prob, dev(psi), prec, T.EVEN,
                                                                                    nrhs=12),
                                                         T.DSLASH_OE, prec, T.RECON18, nrhs=12), prec, T.ODD, 12))
            for k in range(12):
                full = np.zeros((f.prob.volume, 4, 3), dtype=np.complex128)
                full[ev] = psi[k]
                want = -kappa * D.hop_at_sites(f.U, full, dims, BC_AP, od[hs])
                assert rel(outm[k][hs], want) < TOL[prec], (prec, k)
                if k == 0:
                    assert rel(out1[hs], want) < TOL[prec], prec
    finally:
        T.tune_clear()
