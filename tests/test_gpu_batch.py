"""Several lattices in one CG solve (batched grid-stride launches, hipGraph replay).

The batch of the small-lattice configuration (8^4, 12^3 x 24, 16^3 x 32 at
kappa = 0.155, mu = 0.01) is solved with and without graph capture: both must
give bitwise the same solutions, each lattice must match its standalone
tmqcd_cg solve, and the oracle must find every residual <= 1e-10.  The graph is
replayed many times with eager restarts and host synchronisation in between;
the whole solve is repeated to check replays against each other.
"""
import numpy as np
import pytest
import torch

from gpu_util import BC_AP, BC_TWIST, Fields, dev, host, rel
from oracle import dirac as D
from paper_1209_5942_amd import synth
from paper_1209_5942_amd import tmqcd as T

pytestmark = pytest.mark.gpu


def _setup(specs):
    fs, bs = [], []
    for k, (dims, bc) in enumerate(specs):
        f = Fields(dims, 0.4, 300 + k, 0.155, 0.01, bc)
        b = synth.gaussian_spinor(f.prob.volume // 2, 400 + k)
        fs.append(f)
        bs.append(b)
    return fs, bs


def _batch(fs, bs, use_graph, stream=None, **kw):
    probs = [f.prob for f in fs]
    gauges = [f.gauge(T.F64, 0) for f in fs]
    bp = [T.pack_spinor(f.prob, dev(b), T.F64, T.EVEN) for f, b in zip(fs, bs)]
    xs, st, rc = T.cg_batch(probs, gauges, bp, use_graph=use_graph, stream=stream, **kw)
    return [host(T.unpack_spinor(f.prob, x, T.F64, T.EVEN)) for f, x in zip(fs, xs)], st, rc


SPECS = [((8, 8, 8, 8), BC_AP), ((12, 12, 12, 24), BC_AP), ((16, 16, 16, 32), BC_AP)]


@pytest.mark.timeout(300)
def test_batch_graph_equals_eager_and_standalone():
    fs, bs = _setup(SPECS)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        xg, sg, rcg = _batch(fs, bs, True, stream=side)
    side.synchronize()
    xe, se, rce = _batch(fs, bs, False)
    assert rcg == T.OK and rce == T.OK
    for k, f in enumerate(fs):
        assert np.array_equal(xg[k], xe[k]), k
        assert sg[k]["iters"] == se[k]["iters"] and sg[k]["converged"] == 1
        A = lambda v, f=f: D.apply_MhatdagMhat(f.U, v, f.dims, f.kappa, f.mu, f.bc)
        assert D.true_rel_residual(A, bs[k], xg[k]) <= 1e-10
        # the same lattice solved alone
        x1, s1, _ = T.cg(f.prob, {T.F64: f.gauge(T.F64, 0)}, T.pack_spinor(f.prob, dev(bs[k]), T.F64, T.EVEN),
                         tol=1e-10, check_every=8)
        x1 = host(T.unpack_spinor(f.prob, x1, T.F64, T.EVEN))
        assert rel(xg[k], x1) < 1e-12
        assert abs(s1["iters"] - sg[k]["iters"]) <= 1
    # replaying the whole graph solve again gives the same bits
    with torch.cuda.stream(side):
        xg2, _, _ = _batch(fs, bs, True, stream=side)
    side.synchronize()
    for k in range(len(fs)):
        assert np.array_equal(xg[k], xg2[k])


def test_batch_null_stream_graph_and_edge_members():
    """A b = 0 member, a ragged lattice with twisted phases, graph on the null stream."""
    specs = [((4, 4, 4, 4), BC_AP), ((12, 6, 4, 10), BC_TWIST), ((2, 2, 2, 2), BC_TWIST)]
    fs, bs = _setup(specs)
    bs[0] = np.zeros_like(bs[0])
    xs, st, rc = _batch(fs, bs, True)
    assert rc == T.OK
    assert not np.any(xs[0]) and st[0]["converged"] == 1
    for k in (1, 2):
        f = fs[k]
        A = lambda v, f=f: D.apply_MhatdagMhat(f.U, v, f.dims, f.kappa, f.mu, f.bc)
        assert D.true_rel_residual(A, bs[k], xs[k]) <= 1e-10


def test_batch_of_one_and_of_eight():
    fs, bs = _setup([((6, 4, 4, 8), BC_AP)])
    x1, s1, rc = _batch(fs, bs, True)
    assert rc == T.OK and s1[0]["converged"] == 1
    specs = [((4, 4, 4, 4 + 2 * (k % 3)), BC_AP if k % 2 else BC_TWIST) for k in range(8)]
    fs, bs = _setup(specs)
    xs, st, rc = _batch(fs, bs, True)
    assert rc == T.OK
    for k, f in enumerate(fs):
        A = lambda v, f=f: D.apply_MhatdagMhat(f.U, v, f.dims, f.kappa, f.mu, f.bc)
        assert D.true_rel_residual(A, bs[k], xs[k]) <= 1e-10


@pytest.mark.timeout(300)
def test_batch_of_thermal_lattices():
    """Four lattices of short time extent (16^3 x 4, 6, 8 and 20^3 x 4, the bench's thermal batch),
    graph and eager: every member against the oracle, the two bitwise equal."""
    specs = [((16, 16, 16, 4), BC_AP), ((16, 16, 16, 6), BC_AP), ((16, 16, 16, 8), BC_AP), ((20, 20, 20, 4), BC_AP)]
    fs, bs = _setup(specs)
    xg, sg, rcg = _batch(fs, bs, True)
    xe, se, rce = _batch(fs, bs, False)
    assert rcg == T.OK and rce == T.OK
    for k, f in enumerate(fs):
        assert sg[k]["converged"] == 1 and np.array_equal(xg[k], xe[k]), k
        A = lambda v, f=f: D.apply_MhatdagMhat(f.U, v, f.dims, f.kappa, f.mu, f.bc)
        assert D.true_rel_residual(A, bs[k], xg[k]) <= 1e-10


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_member_breakdown_leaves_the_others_solved(use_graph):
    """One lattice's links hold a NaN, so its first p^+ A p is not finite and its solve
    breaks down inside a batched launch; the call reports TMQCD_EBREAKDOWN, and the
    other lattices, whose tiles share those launches, still equal their standalone solves."""
    fs, bs = _setup([((8, 8, 8, 8), BC_AP), ((4, 4, 4, 8), BC_AP), ((12, 12, 12, 24), BC_AP)])
    bad = fs[1].U.copy().reshape(-1, 4, 3, 3)
    bad[5, 2, 0, 0] = np.nan
    probs = [f.prob for f in fs]
    gauges = [f.gauge(T.F64, 0) for f in fs]
    gauges[1] = T.pack_gauge(fs[1].prob, dev(bad))
    bp = [T.pack_spinor(f.prob, dev(b), T.F64, T.EVEN) for f, b in zip(fs, bs)]
    xs, st, rc = T.cg_batch(probs, gauges, bp, use_graph=use_graph, check_every=4, raise_on_breakdown=False)
    assert rc == T.EBREAKDOWN
    assert st[1]["converged"] == 0
    for k in (0, 2):
        f = fs[k]
        x = host(T.unpack_spinor(f.prob, xs[k], T.F64, T.EVEN))
        x1, s1, _ = T.cg(f.prob, {T.F64: f.gauge(T.F64, 0)}, bp[k], tol=1e-10, check_every=4)
        x1 = host(T.unpack_spinor(f.prob, x1, T.F64, T.EVEN))
        assert st[k]["converged"] == 1
        assert rel(x, x1) < 1e-12
        A = lambda v, f=f: D.apply_MhatdagMhat(f.U, v, f.dims, f.kappa, f.mu, f.bc)
        assert D.true_rel_residual(A, bs[k], x) <= 1e-10
