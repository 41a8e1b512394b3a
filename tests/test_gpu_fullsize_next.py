"""Parity at the sizes the bench times for the heatbath and the tree-level Symanzik force.

* One heatbath sweep and one overrelaxation sweep of 24^3 x 48 (beta 5.7, the bench's start
  field and generator streams), on 512 sampled links: a link of direction mu and parity p is
  updated after the links of directions below mu (both parities) and, for p = 1, after the
  parity-0 links of direction mu, so its staple is rebuilt from the fields before and after the
  sweep accordingly and the oracle's single-link update must reproduce the GPU's new link.
* The Symanzik force (c1 = -1/12) on the whole 16^3 x 32 lattice of the bench's HMC set.
"""
import numpy as np
import pytest

from gpu_util import BC_AP, dev, host, rel
from oracle import dirac as D
from oracle import heatbath as OHB
from oracle import symanzik as S
from paper_1209_5942_amd import synth
from paper_1209_5942_amd import tmqcd as T

pytestmark = pytest.mark.gpu


def _site(dims, c):
    return c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]))


def _staple(get, dims, c, mu):
    """Sum of the six Wilson staples of U_mu(c): get(site, direction) returns the link there."""
    dag = lambda m: m.conj().T

    def at(d):
        return _site(dims, [(c[i] + d[i]) % dims[i] for i in range(4)])
    v = np.zeros((3, 3), dtype=np.complex128)
    for nu in range(4):
        if nu == mu:
            continue
        em, en = np.eye(4, dtype=int)[mu], np.eye(4, dtype=int)[nu]
        v += get(at(em), nu) @ dag(get(at(en), mu)) @ dag(get(at(0 * em), nu))
        v += dag(get(at(em - en), nu)) @ dag(get(at(-en), mu)) @ get(at(-en), nu)
    return v


@pytest.mark.timeout(900)
def test_heatbath_and_overrelax_sweeps_24x24x24x48_sampled():
    dims, beta, seed, sweep = (24, 24, 24, 48), 5.7, 92, 1000
    print(f"\nheatbath {dims} sampled links", flush=True)
    prob = T.Problem(dims, 0.15, 0.0, BC_AP)
    U0 = synth.random_links(dims, 0.4, 91)
    g = T.pack_gauge(prob, dev(U0.reshape(-1, 4, 3, 3)))
    T.heatbath(prob, g, beta, seed, sweep)
    U1 = host(T.unpack_gauge(prob, g))
    T.overrelax(prob, g)
    U2 = host(T.unpack_gauge(prob, g))
    coords = D.coords(dims)
    par = coords.sum(axis=1) % 2
    rng = np.random.default_rng(93)
    sites = rng.choice(prob.volume, size=128, replace=False)
    for before, after, hb in ((U0, U1, True), (U1, U2, False)):
        worst = 0.0
        for s in sites:
            for mu in range(4):
                p = par[s]

                def get(site, nu, mu=mu, p=p):
                    new = nu < mu or (nu == mu and p == 1 and par[site] == 0)
                    return (after if new else before)[site, nu]
                V = _staple(get, dims, coords[s], mu)
                want = OHB.update_su3(before[s, mu][None], V[None], beta, seed, np.array([4 * s + mu], dtype=np.uint64),
                                      sweep, hb)[0]
                worst = max(worst, np.abs(after[s, mu] - want).max())
        print(f"{'heatbath' if hb else 'overrelax'}: worst {worst:.2e}", flush=True)
        assert worst < 1e-12


@pytest.mark.timeout(600)
def test_tlsym_force_16x16x16x32_whole_lattice():
    dims = (16, 16, 16, 32)
    print(f"\ntlsym force {dims}", flush=True)
    prob = T.Problem(dims, 0.155, 0.01, BC_AP)
    U = synth.random_links(dims, 0.4, 80)
    g = T.pack_gauge(prob, dev(U.reshape(-1, 4, 3, 3)))
    got = host(T.gauge_force_tlsym(prob, g, 3.9, -1.0 / 12.0))
    assert rel(got, S.force(U, dims, 3.9, -1.0 / 12.0)) < 1e-12
