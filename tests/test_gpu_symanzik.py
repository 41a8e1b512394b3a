"""The tree-level Symanzik gauge force, the rectangle sum and an HMC trajectory with them, on the GPU
against the FP64 oracle (several extents including 2, where rectangles wrap onto themselves)."""
import numpy as np
import pytest

from gpu_util import BC_AP, Fields, dev, host, rel
from oracle import force as F
from oracle import hmc as OH
from oracle import symanzik as S
from paper_1209_5942_amd import hmc as H
from paper_1209_5942_amd import synth
from paper_1209_5942_amd import tmqcd as T

pytestmark = pytest.mark.gpu

C1 = -1.0 / 12.0
DIMS = [(4, 4, 4, 4), (4, 2, 6, 4), (2, 2, 2, 2), (6, 4, 2, 8)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("c1", [C1, 0.3])
def test_tlsym_force_and_rectangles_match_oracle(dims, c1):
    print(f"\ntlsym dims={dims} c1={c1}", flush=True)
    f = Fields(dims, 0.6, 401, 0.155, 0.01, BC_AP)
    g = f.gauge(T.F64, 0)
    want = S.force(f.U, dims, 5.6, c1)
    assert rel(host(T.gauge_force_tlsym(f.prob, g, 5.6, c1)), want) < 1e-12
    p = synth.gaussian_momenta(f.prob.volume, 402)
    pd = dev(p)
    T.gauge_force_tlsym(f.prob, g, 5.6, c1, out=pd, scale=-0.3, accumulate=True)
    assert rel(host(pd), p - 0.3 * want) < 1e-13
    r = float(T.rectangle(f.prob, g)[0])
    assert abs(r - S.rectangle_sum(f.U, dims)) < 1e-12 * 36 * f.prob.volume


@pytest.mark.parametrize("dims", DIMS[:2])
def test_tlsym_at_c1_zero_is_the_wilson_force(dims):
    f = Fields(dims, 0.6, 411, 0.155, 0.01, BC_AP)
    g = f.gauge(T.F64, 0)
    a = host(T.gauge_force_tlsym(f.prob, g, 5.6, 0.0))
    assert rel(a, host(T.gauge_force(f.prob, g, 5.6))) < 1e-13
    assert rel(a, F.gauge_force(f.U, dims, 5.6)) < 1e-12


def test_unit_field_rectangles():
    dims = (4, 4, 2, 2)
    prob = T.Problem(dims, 0.15, 0.0, BC_AP)
    U = np.tile(np.eye(3, dtype=np.complex128), (prob.volume, 4, 1, 1))
    g = T.pack_gauge(prob, dev(U))
    assert float(T.rectangle(prob, g)[0]) == pytest.approx(36.0 * prob.volume, abs=1e-10)
    assert np.abs(host(T.gauge_force_tlsym(prob, g, 6.0, C1))).max() < 1e-14


@pytest.mark.parametrize("n_inner", [1, 2])
def test_eo_2mn_trajectory_with_tlsym_matches_oracle(n_inner):
    dims, kappa, mu, beta = (4, 2, 2, 4), 0.155, 0.01, 5.0
    print(f"\neo 2MN tlsym trajectory n_inner={n_inner}", flush=True)
    f = Fields(dims, 0.4, 421, kappa, mu, BC_AP)
    p = synth.gaussian_momenta(f.prob.volume, 422)
    eta = synth.gaussian_spinor(f.prob.volume // 2, 423)
    n, dt = 4, 0.125
    want = OH.trajectory_eo(f.U, p, eta, 0.5, dims, kappa, mu, BC_AP, beta, n, dt, n_inner, c1=C1)
    h = H.HMC(f.prob, f.U_dev, beta, tol=1e-14, eo=True, c1=C1)
    pd = dev(p)
    out = h.trajectory(pd, dev(eta), 0.5, n, dt, integrator="2mn", n_inner=n_inner)
    assert abs(out["H0"] - want["H0"]) < 1e-10 * abs(want["H0"])
    assert abs(out["dH"] - want["dH"]) < 1e-8, (out["dH"], want["dH"])
    assert out["accepted"] == want["accepted"]
    assert np.abs(host(pd) - want["p_proposed"]).max() < 1e-9
    got_u = host(T.unpack_gauge(f.prob, h.U))
    assert np.abs(got_u - (want["U_proposed"] if out["accepted"] else f.U)).max() < 1e-10
