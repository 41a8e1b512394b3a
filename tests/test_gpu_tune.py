"""The autotuner: every admitted launch shape reproduces the default shape's output bitwise,
tuned launches give the same operator and solver results, and the table round-trips through a file."""
import json

import numpy as np
import pytest

from gpu_util import BC_AP, BC_TWIST, Fields, dev, host
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
        assert r["candidates"] == 4 and r["rejected"] == 0
        assert r["block"] in (128, 256) and r["swizzle"] in (0, 1) and 0 < r["us"] <= r["default_us"] * 1.0001
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
