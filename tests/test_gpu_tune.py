"""The autotuner: every admitted launch shape reproduces the default shape's output bitwise,
tuned launches give the same operator and solver results, the table round-trips through a file,
and every pinned launch shape (block size x block order) matches the oracle."""
import json

import numpy as np
import pytest

from gpu_util import BC_AP, BC_TWIST, TOL, Fields, dev, host, oracle_op, rel
from oracle import dirac as D
from paper_1209_5942_amd import synth
from paper_1209_5942_amd import tmqcd as T

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,recon", [(T.F64, T.RECON18), (T.F32, T.RECON12), (T.F16, T.RECON18)])
def test_tune_admits_bitwise_equal_shapes_and_keeps_results(tmp_path, prec, recon):
    f = Fields((12, 6, 4, 10), 0.5, 501, 0.16, 0.005, BC_TWIST)
    g = f.gauge(prec, recon)
    psi = f.spinor(T.EVEN, 502)
    inp = T.pack_spinor(f.prob, dev(psi), prec, T.EVEN)
    T.tune_clear()
    before = host(T.unpack_spinor(f.prob, T.dslash(f.prob, g, inp, T.MHATDAGMHAT, prec, recon), prec, T.EVEN))
    res = T.tune(f.prob, g, prec, recon)
    assert [r["kernel_class"] for r in res] == [0, 1, 2]
    for r in res:
        assert r["candidates"] == 12 and r["rejected"] == 0
        assert r["block"] in (128, 256) and r["order"] in range(6) and 0 < r["us"] <= r["default_us"] * 1.0001
    after = host(T.unpack_spinor(f.prob, T.dslash(f.prob, g, inp, T.MHATDAGMHAT, prec, recon), prec, T.EVEN))
    assert np.array_equal(before, after)
    path = tmp_path / "tune.jsonl"
    T.tune_save(path)
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert len(lines) == 3 and all(l["dims"] == [12, 6, 4, 10] and l["prec"] == prec for l in lines)
    T.tune_clear()
    T.tune_load(path)
    again = host(T.unpack_spinor(f.prob, T.dslash(f.prob, g, inp, T.MHATDAGMHAT, prec, recon), prec, T.EVEN))
    assert np.array_equal(before, again)
    T.tune_clear()


def test_tuned_cg_matches_untuned():
    f = Fields((16, 8, 8, 16), 0.5, 511, 0.16, 0.005, BC_AP)
    b = T.pack_spinor(f.prob, dev(synth.gaussian_spinor(f.prob.volume // 2, 512)), T.F64, T.EVEN)
    T.tune_clear()
    x0, s0, _ = T.cg(f.prob, {T.F64: f.gauge(T.F64, 0)}, b, tol=1e-10)
    T.tune(f.prob, f.gauge(T.F64, 0))
    x1, s1, _ = T.cg(f.prob, {T.F64: f.gauge(T.F64, 0)}, b, tol=1e-10)
    T.tune_clear()
    assert s0["iters"] == s1["iters"]
    a0 = host(T.unpack_spinor(f.prob, x0, T.F64, T.EVEN))
    a1 = host(T.unpack_spinor(f.prob, x1, T.F64, T.EVEN))
    # block size changes only the order of the FP64 partial sums of the reductions
    assert np.linalg.norm(a1 - a0) <= 1e-12 * np.linalg.norm(a0)


SHAPES = [(b, o) for b in (128, 256) for o in range(6)]


@pytest.mark.parametrize("block,order", SHAPES)
@pytest.mark.parametrize("dims,bc", [((12, 6, 4, 10), BC_TWIST), ((2, 4, 6, 8), BC_AP)])
def test_pinned_shapes_match_oracle(block, order, dims, bc):
    """Every block order covers each output site once, on ragged lattices, for one and two parities."""
    f = Fields(dims, 0.5, 521, 0.16, 0.02, bc)
    try:
        T.tune_clear()
        for prec in (T.F64, T.F32):
            for cls in (0, 1, 2):
                T.tune_set(f.prob, prec, T.RECON18, cls, block, order)
        for op, sub_in, sub_out in [(T.MHATDAGMHAT, T.EVEN, T.EVEN), (T.M, T.FULL, T.FULL),
                                    (T.DSLASH_OE, T.EVEN, T.ODD)]:
            psi = f.spinor(sub_in, 522)
            want = oracle_op(op, f.U, psi, f.dims, f.kappa, f.mu, f.bc)
            for prec in (T.F64, T.F32):
                out = T.dslash(f.prob, f.gauge(prec, T.RECON18), T.pack_spinor(f.prob, dev(psi), prec, sub_in), op,
                               prec, T.RECON18)
                got = host(T.unpack_spinor(f.prob, out, prec, sub_out))
                assert rel(got, want) <= 4 * TOL[prec], (op, prec)
        b = synth.gaussian_spinor(f.prob.volume // 2, 523)
        for inner in (T.F64, T.F32):
            g = {T.F64: f.gauge(T.F64, T.RECON18), inner: f.gauge(inner, T.RECON18)}
            x, st, rc = T.cg(f.prob, g, T.pack_spinor(f.prob, dev(b), T.F64, T.EVEN), tol=1e-10, inner_prec=inner)
            assert rc == T.OK and st["converged"] == 1
            xs = host(T.unpack_spinor(f.prob, x, T.F64, T.EVEN))
            A = lambda v: D.apply_MhatdagMhat(f.U, v, f.dims, f.kappa, f.mu, f.bc)
            assert D.true_rel_residual(A, b, xs) <= 1e-10
    finally:
        T.tune_clear()


@pytest.mark.parametrize("order,group", [(0, 0), (1, 0), (2, 0), (3, 0), (4, 0), (5, 0), (2, 5), (3, 4), (4, 5)])
@pytest.mark.parametrize("dims,bc", [((12, 6, 4, 10), BC_TWIST), ((4, 4, 8, 8), BC_AP)])
def test_pinned_multi_rhs_orders_match_oracle(order, group, dims, bc):
    """The multi-RHS kernel in every block order and with rhs groups (5 per block: 5 + 5 + 2): 12 Gaussian
    fields through M (both parities) and Mhat^dag Mhat."""
    f = Fields(dims, 0.5, 531, 0.16, 0.02, bc)
    try:
        T.tune_clear()
        for prec in (T.F64, T.F32):
            T.tune_set(f.prob, prec, T.RECON18, 3, 256, order, nrhs=12, group=group)
        for op in (T.M, T.MHATDAGMHAT):
            sub_in, sub_out = T.OP_SUBSETS[op]
            src = f.spinor(sub_in, 532 + op, nrhs=12)
            for prec in (T.F64, T.F32):
                inp = T.pack_spinor(f.prob, dev(src), prec, sub_in, nrhs=12)
                out = host(T.unpack_spinor(f.prob, T.dslash(f.prob, f.gauge(prec, 0), inp, op, prec, 0, nrhs=12),
                                           prec, sub_out, 12))
                for k in range(12):
                    want = oracle_op(op, f.U, src[k], f.dims, f.kappa, f.mu, f.bc)
                    assert rel(out[k], want) <= 4 * TOL[prec], (op, prec, k)
    finally:
        T.tune_clear()


def test_tune_mrhs_admits_equal_orders_and_keeps_results():
    f = Fields((12, 6, 4, 10), 0.5, 541, 0.16, 0.005, BC_TWIST)
    psi = f.spinor(T.EVEN, 542, nrhs=12)
    inp = T.pack_spinor(f.prob, dev(psi), T.F64, T.EVEN, nrhs=12)
    g = f.gauge(T.F64, 0)
    try:
        T.tune_clear()
        # compare the sites only: the packed fields' padding (this lattice's half volume is not a
        # multiple of 64) is never written
        before = host(T.unpack_spinor(f.prob, T.dslash(f.prob, g, inp, T.MHATDAGMHAT, nrhs=12), T.F64, T.EVEN,
                                      nrhs=12))
        r = T.tune_mrhs(f.prob, g, 12)
        assert r["kernel_class"] == 3 and r["candidates"] == 18 and r["rejected"] == 0
        assert r["block"] == 256 and r["order"] in range(6) and r["group"] in (0, 6, 4)
        assert 0 < r["us"] <= r["default_us"] * 1.0001
        after = host(T.unpack_spinor(f.prob, T.dslash(f.prob, g, inp, T.MHATDAGMHAT, nrhs=12), T.F64, T.EVEN,
                                     nrhs=12))
        assert np.array_equal(before, after)
    finally:
        T.tune_clear()
