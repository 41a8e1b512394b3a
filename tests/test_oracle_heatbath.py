"""Pins for the oracle's heatbath and overrelaxation (no GPU).

* The x0 sampler against the exact distribution sqrt(1 - x0^2) exp(alpha x0)
  (Kolmogorov-Smirnov, both methods and the switch between them, alpha = 0).
* The SU(3) update as a Markov chain for one link with staple sum c 1: its
  stationary mean of Re Tr U / 3 against the exact value under the weight
  exp((beta c / 3) Re Tr U), computed from Weyl's integration formula over the
  eigenphases.
* beta = 0: one sweep gives Haar-distributed links (<Tr U> = 0, <|Tr U|^2> = 1).
* Overrelaxation keeps Re Tr[U V] of every link and the plaquette sum exactly,
  and links stay in SU(3).
* The strong-coupling plaquette <Re Tr P / 3> = beta / 18 + O(beta^2) on 4^4.
* The generator: uniformity, bit balance, and decorrelation of neighbouring
  counters and keys (statistical pins of the Philox implementation).
"""
import numpy as np
import pytest

from oracle import force as F
from oracle import heatbath as HB
from paper_1209_5942_amd import synth


def _x0_cdf(alpha, grid):
    x = np.linspace(-1.0, 1.0, 200001)
    d = np.sqrt(np.maximum(0.0, 1.0 - x * x)) * np.exp(alpha * (x - 1.0))
    c = np.concatenate([[0.0], np.cumsum(0.5 * (d[1:] + d[:-1]) * np.diff(x))])
    return np.interp(grid, x, c / c[-1])


@pytest.mark.parametrize("alpha", [0.0, 0.7, 1.99, 2.0, 6.0, 30.0])
def test_x0_sampler_distribution(alpha):
    n = 50000
    link = np.arange(n, dtype=np.uint64)
    x0 = np.sort(HB.sample_x0(np.full(n, alpha), 77, link, 3, 1))
    emp = np.arange(1, n + 1) / n
    d = np.max(np.abs(emp - _x0_cdf(alpha, x0)))
    assert d < 1.63 / np.sqrt(n), d


def _weyl_mean_retr(gamma, m=400):
    """<Re Tr U / 3> under exp(gamma Re Tr U) dU on SU(3), by Weyl's integration formula."""
    t = 2.0 * np.pi * np.arange(m) / m
    t1, t2 = np.meshgrid(t, t, indexing="ij")
    z = np.stack([np.exp(1j * t1), np.exp(1j * t2), np.exp(-1j * (t1 + t2))])
    vdm = np.abs(z[0] - z[1]) ** 2 * np.abs(z[0] - z[2]) ** 2 * np.abs(z[1] - z[2]) ** 2
    tr = z.sum(axis=0).real
    w = vdm * np.exp(gamma * tr)
    return float((w * tr).sum() / w.sum() / 3.0)


@pytest.mark.parametrize("beta,c", [(6.0, 1.0), (3.0, 0.5), (9.0, 1.0)])
def test_single_link_chain_matches_weyl_integral(beta, c):
    n, sweeps, skip = 20000, 30, 15
    u = np.tile(np.eye(3, dtype=np.complex128), (n, 1, 1))
    V = np.tile(c * np.eye(3, dtype=np.complex128), (n, 1, 1))
    link = np.arange(n, dtype=np.uint64)
    acc = []
    for sw in range(sweeps):
        u = HB.update_su3(u, V, beta, 2024, link, sw, True)
        if sw >= skip:
            acc.append(np.trace(u, axis1=1, axis2=2).real / 3.0)
    per_link = np.mean(acc, axis=0)          # links are independent; sweeps of one link are not
    mean, err = per_link.mean(), per_link.std(ddof=1) / np.sqrt(n)
    want = _weyl_mean_retr(beta * c / 3.0)
    assert abs(mean - want) < 5 * err + 2e-3, (mean, want, err)
    np.testing.assert_allclose(np.linalg.det(u), 1.0, atol=1e-13)


def test_beta_zero_gives_haar_links():
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 0.2, 7)
    U1 = HB.heatbath_sweep(U, dims, 0.0, 99, 0)
    tr = np.trace(U1, axis1=-2, axis2=-1).reshape(-1)
    assert abs(tr.mean()) < 4 / np.sqrt(tr.size)
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 4 * np.sqrt(2.0 / tr.size)


def test_overrelaxation_is_microcanonical():
    rng = np.random.default_rng(8)
    n = 500
    u = synth.random_links((2, 2, 5, 10), 0.8, 9).reshape(-1, 3, 3)[:n]
    V = rng.normal(size=(n, 3, 3)) + 1j * rng.normal(size=(n, 3, 3))
    u1 = HB.update_su3(u, V, 0.0, 0, np.arange(n, dtype=np.uint64), 0, False)
    before = np.trace(u @ V, axis1=1, axis2=2).real
    after = np.trace(u1 @ V, axis1=1, axis2=2).real
    np.testing.assert_allclose(after, before, rtol=0, atol=1e-12)
    assert np.abs(u1 - u).max() > 0.1
    dims = (4, 4, 2, 4)
    U = synth.random_links(dims, 0.6, 10)
    U2 = HB.overrelax_sweep(U, dims)
    assert abs(F.plaquette_sum(U2, dims) - F.plaquette_sum(U, dims)) < 1e-10
    np.testing.assert_allclose(np.linalg.det(U2), 1.0, atol=1e-13)
    np.testing.assert_allclose(U2 @ np.conj(np.swapaxes(U2, -1, -2)), np.broadcast_to(np.eye(3), U2.shape),
                               atol=1e-13)


def test_strong_coupling_plaquette():
    dims, beta = (4, 4, 4, 4), 0.3
    U = synth.random_links(dims, 0.3, 11)
    vals = []
    for sw in range(40):
        U = HB.heatbath_sweep(U, dims, beta, 5, sw)
        if sw >= 5:
            vals.append(F.plaquette_sum(U, dims) / (6 * int(np.prod(dims))) / 3.0)
    assert abs(np.mean(vals) - beta / 18.0) < 0.004, np.mean(vals)


def test_generator_statistics():
    n = 1 << 16
    c0 = np.arange(n, dtype=np.uint64)
    w = HB.philox4x32(c0, 0, 0, 0, 12345, 678)
    words = np.concatenate(w)
    u = HB.uniform(words)
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / u.size)
    hist = np.bincount((u * 64).astype(int), minlength=64)
    chi2 = np.sum((hist - u.size / 64) ** 2 / (u.size / 64))
    assert chi2 < 110, chi2                     # 63 degrees of freedom: p < 1e-4 above this
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint64)) & np.uint64(1)).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 4 * 0.5 / np.sqrt(words.size))
    # neighbouring counters and neighbouring keys give uncorrelated streams
    u0 = HB.uniform(w[0])
    assert abs(np.corrcoef(u0[:-1], u0[1:])[0, 1]) < 4 / np.sqrt(n)
    w_k = HB.philox4x32(c0, 0, 0, 0, 12346, 678)
    assert abs(np.corrcoef(u0, HB.uniform(w_k[0]))[0, 1]) < 4 / np.sqrt(n)
    # one flipped key bit changes about half of the output bits
    flips = np.unpackbits((w[0] ^ w_k[0]).astype(">u4").view(np.uint8)).reshape(n, 32).sum(axis=1)
    assert abs(flips.mean() - 16.0) < 0.1


def test_decision_hooks_record_margins_and_flip_outcomes():
    """The sampler's test hooks: every watched decision's margin has the sign of the outcome
    taken (the accepted trial >= 0, the rejected ones < 0), and flipping the acceptance of
    the accepted trial moves x0 to a later trial."""
    alpha = np.array([0.7, 3.5, 1.9, 6.0])
    link = np.array([11, 12, 13, 14], dtype=np.uint64)
    watch = {int(l): [] for l in link}
    x0 = HB.sample_x0(alpha, 99, link, 5, 1, watch=watch)
    for i, l in enumerate(link):
        recs = watch[int(l)]
        assert recs[0][0] == (int(l), 1, -1) and (recs[0][1] > 0) == (alpha[i] < 2)
        trials = recs[1:]
        assert all(m < 0 for _, m in trials[:-1]) and trials[-1][1] >= 0
        last = trials[-1][0]
        x1 = HB.sample_x0(alpha, 99, link, 5, 1, flips={last})
        assert np.array_equal(np.delete(x1, i), np.delete(x0, i))
        assert x1[i] != x0[i]
    # the method switch taken the other way also changes the sample
    x2 = HB.sample_x0(alpha, 99, link, 5, 1, flips={(13, 1, -1)})
    assert x2[2] != x0[2] and np.array_equal(np.delete(x2, 2), np.delete(x0, 2))
