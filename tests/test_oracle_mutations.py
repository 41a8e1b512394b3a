"""Each plausible mistake planted in the oracle must be caught by at least one pin.

The mistakes are planted by patching the oracle module for the duration of one
test (on the CPU); the pins are the closed-form / invariant / brute-force checks
of test_oracle_operator and test_oracle_force_hmc, called unchanged.
"""
import numpy as np
import pytest

import test_oracle_force_hmc as PF
import test_oracle_operator as PO
from oracle import dirac as D
from oracle import force as F

OPERATOR_PINS = [
    lambda: PO.test_free_field_spectrum_M_2x2x2x2(0.15, 0.01),
    PO.test_free_field_massless_at_kappa_one_eighth,
    PO.test_dense_block_matrix_2x2x2x2,
    PO.test_sparse_block_matrix_distinct_extents,
    PO.test_gamma5_hermiticity_random_field,
    PO.test_twisted_mass_shift_identity,
    PO.test_gauge_covariance,
]


def _caught(pins):
    for pin in pins:
        try:
            pin()
        except AssertionError:
            return True
    return False


MUTATIONS = {
    # (1 + gamma) where (1 - gamma) belongs, and vice versa
    "projector sign": lambda mp: mp.setattr(D, "GAMMA", -D.GAMMA),
    # boundary phases dropped
    "boundary phase": lambda mp: mp.setattr(D, "_scale_slice", lambda a, axis, index, factor: None),
    # x and t axes confused in the lattice view
    "axis order": lambda mp: mp.setattr(D, "AXIS", (0, 1, 2, 3)),
    # twist with the wrong sign of mu
    "twist sign": lambda mp: mp.setattr(D, "twist", (lambda f: (lambda psi, kappa, mu: f(psi, kappa, -mu)))(D.twist)),
    # the printed kappa/2 prefactor taken literally
    "kappa/2": lambda mp: mp.setattr(D, "hop", (lambda h: (lambda *a, **k: 0.5 * h(*a, **k)))(D.hop)),
    # gamma5 replaced by the identity
    "gamma5": lambda mp: mp.setattr(D, "GAMMA5", np.eye(4, dtype=np.complex128)),
    # forward neighbour taken from x - mu (roll in the wrong direction)
    "neighbour direction": lambda mp: mp.setattr(D.np, "roll", (lambda r: (lambda a, s, axis: r(a, -s, axis)))(np.roll)),
}


def test_unmutated_oracle_passes_every_pin():
    assert not _caught(OPERATOR_PINS)


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_operator_mistake_fails_a_pin(monkeypatch, name):
    MUTATIONS[name](monkeypatch)
    assert _caught(OPERATOR_PINS), f"no pin caught the planted mistake: {name}"


FORCE_MUTATIONS = {
    "force sign": lambda mp: mp.setattr(F, "fermion_force",
                                        (lambda f: (lambda *a, **k: -f(*a, **k)))(F.fermion_force)),
    "force factor": lambda mp: mp.setattr(F, "fermion_force",
                                          (lambda f: (lambda *a, **k: 0.5 * f(*a, **k)))(F.fermion_force)),
    "spin projectors dropped": lambda mp: mp.setattr(F, "GAMMA", 0.0 * F.GAMMA),
    "gauge force sign": lambda mp: mp.setattr(F, "gauge_force",
                                              (lambda f: (lambda *a, **k: -f(*a, **k)))(F.gauge_force)),
}


@pytest.mark.parametrize("name", list(FORCE_MUTATIONS))
def test_planted_force_mistake_fails_a_pin(monkeypatch, name):
    FORCE_MUTATIONS[name](monkeypatch)
    pins = [lambda: PF.test_fermion_force_vs_finite_differences(PF.BC), PF.test_gauge_force_vs_finite_differences]
    assert _caught(pins), f"no pin caught the planted mistake: {name}"
