"""Each plausible mistake planted in the oracle must be caught by at least one pin.

The mistakes are planted by patching the oracle module for the duration of one
test (on the CPU); the pins are the closed-form / invariant / brute-force checks
of test_oracle_operator and test_oracle_force_hmc, called unchanged.
"""
import numpy as np
import pytest

import test_oracle_eo_hmc as PE
import test_oracle_force_hmc as PF
import test_oracle_operator as PO
from oracle import dirac as D
from oracle import force as F
from oracle import hmc as H

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


def _eo_force_with(y_odd=1.0, y_mu_sign=-1.0, y_kappa=True, x_odd_dag=False):
    """The even-odd force with one planted change to how the odd halves or the kappa factor are formed."""
    def f(U, X_e, dims, kappa, mu, bc):
        y_e = D.apply_Mhat(U, X_e, dims, kappa, mu, bc)
        x_o = D.twist_inv(D.hop_pq(U, X_e, dims, bc, 1, dagger=x_odd_dag), kappa, mu)
        y_o = D.twist_inv(D.hop_pq(U, y_e, dims, bc, 1, dagger=True), kappa, y_mu_sign * mu)
        x = D.to_full(X_e, dims, 0) + D.to_full(x_o, dims, 1)
        y = D.to_full(y_e, dims, 0) + y_odd * D.to_full(y_o, dims, 1)
        return F.fermion_force(U, x, (kappa if y_kappa else 1.0) * y, dims, kappa, bc)
    return f


EO_FORCE_MUTATIONS = {
    "odd half of Y dropped": dict(y_odd=0.0),
    "Y_o with A(mu)^-1 in place of A(-mu)^-1": dict(y_mu_sign=1.0),
    "kappa factor on Y dropped": dict(y_kappa=False),
    "X_o from the daggered hop": dict(x_odd_dag=True),
}


def test_unmutated_eo_force_copy_passes():
    import unittest.mock as um
    with um.patch.object(F, "fermion_force_eo", _eo_force_with()):
        PE.test_eo_force_vs_finite_differences(PE.BC_TWIST, 0.2, PE.SITES[:2])


@pytest.mark.parametrize("name", list(EO_FORCE_MUTATIONS))
def test_planted_eo_force_mistake_fails_a_pin(monkeypatch, name):
    monkeypatch.setattr(F, "fermion_force_eo", _eo_force_with(**EO_FORCE_MUTATIONS[name]))
    pins = [lambda: PE.test_eo_force_vs_finite_differences(PE.BC_TWIST, 0.2, PE.SITES[:2])]
    assert _caught(pins), f"no pin caught the planted mistake: {name}"


def _omelyan_with(w_mid):
    """2MN with the middle fermion-force weight replaced by w_mid(lam) (the scheme needs 1 - 2 lam)."""
    def integ(U, p, grad_outer, grad_inner, n_outer, dt, n_inner=1, lam=H.LAMBDA_2MN):
        def inner(u, q, tau):
            if grad_inner is None:
                return H.su3_exp(q, tau) @ u, q
            h = tau / n_inner
            for _ in range(n_inner):
                q = q - lam * h * grad_inner(u)
                u = H.su3_exp(q, 0.5 * h) @ u
                q = q - w_mid(lam) * h * grad_inner(u)
                u = H.su3_exp(q, 0.5 * h) @ u
                q = q - lam * h * grad_inner(u)
            return u, q
        u, q = U.copy(), p.copy()
        for _ in range(n_outer):
            q = q - lam * dt * grad_outer(u)
            u, q = inner(u, q, 0.5 * dt)
            q = q - w_mid(lam) * dt * grad_outer(u)
            u, q = inner(u, q, 0.5 * dt)
            q = q - lam * dt * grad_outer(u)
        return u, q
    return integ


@pytest.mark.parametrize("w_mid", [lambda lam: 1.0 - 2.0 * lam, lambda lam: 1.0 - lam, lambda lam: 2.0 * lam])
def test_planted_2mn_weight_mistake_fails_a_pin(monkeypatch, w_mid):
    monkeypatch.setattr(H, "omelyan", _omelyan_with(w_mid))
    caught = _caught([lambda: PE.test_omelyan_energy_error_is_second_order(3)])
    assert caught == (abs(2.0 * H.LAMBDA_2MN + w_mid(H.LAMBDA_2MN) - 1.0) > 1e-12), "the dt^2 pin must fail exactly when the weights do not sum to one"


import test_oracle_symanzik as PS
from oracle import symanzik as S


def _rect_paths_swapped_side():
    paths = {mu: [list(p) for p in ps] for mu, ps in S.RECTANGLE_STAPLE_PATHS.items()}
    s, m = paths[1][1][0], 2
    paths[1][1] = [-s, -m, -m, s, m]     # the second-link rectangle on the wrong side (still a closed loop)
    return paths


SYMANZIK_MUTATIONS = {
    "rectangles long in the first direction only": lambda mp: mp.setattr(
        S, "rectangle_sum", lambda U, dims: sum(
            S.loop_trace_sum(U, dims, [m + 1, m + 1, n + 1, -(m + 1), -(m + 1), -(n + 1)])
            for m in range(4) for n in range(m + 1, 4)) * 2),
    "rectangles as 1x1 loops": lambda mp: mp.setattr(
        S, "rectangle_sum", lambda U, dims: 2 * S.plaquette_sum(U, dims)),
    "c1 sign flipped in the action": lambda mp: mp.setattr(
        S, "action", (lambda f: (lambda U, dims, beta, c1: f(U, dims, beta, -c1)))(S.action)),
    "c0 = 1 + 8 c1": lambda mp: mp.setattr(
        S, "action", lambda U, dims, beta, c1: float(beta / 3.0 * (
            (1 + 8 * c1) * (18.0 * int(np.prod(dims)) - S.plaquette_sum(U, dims))
            + c1 * (36.0 * int(np.prod(dims)) - S.rectangle_sum(U, dims))))),
    "rectangle staple on the wrong side": lambda mp: mp.setattr(S, "RECTANGLE_STAPLE_PATHS",
                                                                _rect_paths_swapped_side()),
}


@pytest.mark.parametrize("name", list(SYMANZIK_MUTATIONS))
def test_planted_symanzik_mistake_fails_a_pin(monkeypatch, name):
    SYMANZIK_MUTATIONS[name](monkeypatch)
    pins = [lambda: PS.test_abelian_plane_wave_closed_form(0.3), PS.test_tree_level_improvement_fixes_the_sign_of_c1,
            PS.test_unit_field, lambda: PS.test_force_vs_finite_differences(0.2)]
    assert _caught(pins), f"no pin caught the planted mistake: {name}"


import test_oracle_bicgstab as PB
from oracle import bicgstab as BI


def _bicgstab_with(beta_ratio=True, omega_conj=False):
    """BiCGStab with one planted change: beta without the alpha/omega factor, or omega from (s, t)."""
    def solve(apply_A, b, tol=1e-10, maxiter=400, x0=None):
        x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128, copy=True)
        r = b - apply_A(x) if x0 is not None else b.copy()
        rt = r.copy()
        bb = np.vdot(b, b).real
        if bb == 0.0:
            return np.zeros_like(b), 0, True
        rho_prev = alpha = omega = 1.0 + 0.0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        k = 0
        while np.vdot(r, r).real > tol * tol * bb:
            if k >= maxiter:
                return x, k, False
            rho = np.vdot(rt, r)
            beta = (rho / rho_prev) * ((alpha / omega) if beta_ratio else 1.0)
            p = r + beta * (p - omega * v)
            v = apply_A(p)
            alpha = rho / np.vdot(rt, v)
            s = r - alpha * v
            t = apply_A(s)
            omega = (np.vdot(s, t) if omega_conj else np.vdot(t, s)) / np.vdot(t, t).real
            x = x + alpha * p + omega * s
            r = s - omega * t
            rho_prev = rho
            k += 1
        return x, k, True
    return solve


@pytest.mark.parametrize("kw", [dict(beta_ratio=False), dict(omega_conj=True)])
def test_planted_bicgstab_mistake_fails_a_pin(monkeypatch, kw):
    monkeypatch.setattr(BI, "bicgstab", _bicgstab_with(**kw))
    pins = [PB.test_small_nonsymmetric_matrix_against_lu,
            lambda: PB.test_M_against_dense_lu((4, 2, 2, 4), 0.16, 0.3)]
    assert _caught(pins), f"no pin caught the planted mistake: {kw}"


def test_unplanted_bicgstab_copy_passes(monkeypatch):
    monkeypatch.setattr(BI, "bicgstab", _bicgstab_with())
    PB.test_small_nonsymmetric_matrix_against_lu()
    PB.test_M_against_dense_lu((4, 2, 2, 4), 0.16, 0.3)


import test_oracle_heatbath as PH
from oracle import heatbath as HBO


HEATBATH_MUTATIONS = {
    # alpha = beta k (the 2/3 of the normalisation lost)
    "alpha factor": lambda mp: mp.setattr(HBO, "sample_x0", (lambda f: (lambda alpha, *a, **k: f(
        1.5 * np.asarray(alpha), *a, **k)))(HBO.sample_x0)),
    # sign of a2 in the quaternion projection
    "projection sign": lambda mp: mp.setattr(HBO, "su2_project", (lambda f: (lambda w: (lambda q: (
        q[0], q[1], -q[2], q[3]))(f(w))))(HBO.su2_project)),
    # the accepted x0 reflected: weight exp(-alpha x0)
    "x0 sign": lambda mp: mp.setattr(HBO, "sample_x0", (lambda f: (lambda *a, **k: -f(*a, **k)))(HBO.sample_x0)),
}


@pytest.mark.parametrize("name", list(HEATBATH_MUTATIONS))
def test_planted_heatbath_mistake_fails_a_pin(monkeypatch, name):
    HEATBATH_MUTATIONS[name](monkeypatch)
    pins = [lambda: PH.test_single_link_chain_matches_weyl_integral(6.0, 1.0), PH.test_overrelaxation_is_microcanonical]
    assert _caught(pins), f"no pin caught the planted mistake: {name}"
