"""FP64 oracle for the pseudofermion action, its link gradient, and the Wilson gauge action.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.

* Pseudofermion action (paper, section 2.2 and the HMC paragraph): for two
  flavours S_f = phi^dag (M^dag M)^{-1} phi.
* Link parametrisation: U_mu(x) -> exp(i w^a T^a) U_mu(x), T^a = lambda^a / 2;
  the gradient G^a_mu(x) = dS/dw^a at w = 0.  The HMC force is F = -G.
* Fermion force (paper, the identity for the derivative of D^{-1}; the printed
  identity lacks the minus sign of d(D^{-1}) = -D^{-1} (dD) D^{-1}): with
  X = (M^dag M)^{-1} phi and Y = M X, dS_f = -2 Re(Y^dag dM X) and dM = -kappa dH,
  since the twisted diagonal does not depend on U.  Written out per link:
      G^a = -2 kappa Im Tr_c[ T^a ( b+ Q1 - conj(b+) Q2 ) ]
      Q1  = sum_spin [(1 - gamma_mu) U_mu(x) X(x+mu)] (x) Y(x)^dag
      Q2  = sum_spin X(x) (x) [U_mu(x) (1 + gamma_mu) Y(x+mu)]^dag
* Even-odd pseudofermion action (the paper's even-odd preconditioning applied to
  the HMC): det(M^dag M) = det(A^dag A)_oo det(Mhat^dag Mhat), and the first
  factor does not depend on U, so the two-flavour action may be taken as
  S_f^eo = phi_e^dag (Mhat^dag Mhat)^{-1} phi_e on even sites.  Only the hops in
  Mhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe depend on U:
      dMhat = -kappa^2 (dH_eo A^{-1} H_oe + H_eo A^{-1} dH_oe),
  so with X_e = (Mhat^dag Mhat)^{-1} phi_e, Y_e = Mhat X_e, X_o = A^{-1} H_oe X_e
  and Y_o = A^{-dag} (H_eo)^dag Y_e,
      dS = -2 Re(Y_e^dag dMhat X_e) = 2 kappa^2 Re(Y_e^dag dH_eo X_o + Y_o^dag dH_oe X_e),
  which is the full-lattice form 2 kappa Re(Y^dag dH X) for the full fields
  X = (X_e, X_o) and Y = kappa (Y_e, Y_o): the same per-link formula.
* Gauge action: the paper's tree-level Symanzik action with c1 = 0 (its
  unimproved limit), normalised S_g = (beta/3) sum_{x, mu<nu} (3 - Re Tr P_mu_nu(x)).
  Its gradient is G^a = (beta/3) Im Tr[T^a U_mu(x) V_mu(x)] with V_mu(x) the sum
  of the six staples.  No boundary phases enter S_g.
"""
from __future__ import annotations

import numpy as np

from .dirac import (AXIS, GAMMA, ID4, apply_MdagM, apply_Mhat, apply_MhatdagMhat, cg, hop_pq, shape4, to_full,
                    twist_inv)

__all__ = ["T_GEN", "fermion_force", "fermion_action", "fermion_action_eo", "fermion_force_eo", "plaquette_sum",
           "gauge_action", "gauge_force", "staple_sum"]


def _gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda^a (the standard su(3) basis), entry by entry.

    lambda^1..3 embed the Pauli matrices in the (0, 1) block, lambda^4, lambda^5 the
    x and y Pauli matrices in the (0, 2) rows and columns, lambda^6, lambda^7 those
    in (1, 2), and lambda^8 = diag(1, 1, -2) / sqrt(3).  Pinned by the tests: every
    one hermitian and traceless, Tr(lambda^a lambda^b) = 2 delta^ab, and the
    structure constants f^123 = 1, f^458 = f^678 = sqrt(3)/2 of
    [T^a, T^b] = i f^abc T^c.
    """
    s3 = 1.0 / np.sqrt(3.0)
    lam = np.array([
        [[0, 1, 0], [1, 0, 0], [0, 0, 0]],
        [[0, -1j, 0], [1j, 0, 0], [0, 0, 0]],
        [[1, 0, 0], [0, -1, 0], [0, 0, 0]],
        [[0, 0, 1], [0, 0, 0], [1, 0, 0]],
        [[0, 0, -1j], [0, 0, 0], [1j, 0, 0]],
        [[0, 0, 0], [0, 0, 1], [0, 1, 0]],
        [[0, 0, 0], [0, 0, -1j], [0, 1j, 0]],
        [[s3, 0, 0], [0, s3, 0], [0, 0, -2 * s3]],
    ], dtype=np.complex128)
    return lam


# su(3) generators T^a = lambda^a / 2 (the link parametrisation exp(i w^a T^a) U)
T_GEN = _gell_mann() / 2


def _bplus(dims, mu, bc) -> np.ndarray:
    b = np.ones(shape4(dims), dtype=np.complex128)
    sl = [slice(None)] * 4
    sl[AXIS[mu]] = int(dims[mu]) - 1
    b[tuple(sl)] = complex(bc[mu])
    return b


def fermion_force(U, X, Y, dims, kappa, bc) -> np.ndarray:
    """dS_f/dw^a for every link, shape (V, 4, 8), from X = (M^dag M)^{-1} phi and Y = M X."""
    sh = shape4(dims)
    u = U.reshape(sh + (4, 3, 3))
    x = X.reshape(sh + (4, 3))
    y = Y.reshape(sh + (4, 3))
    g = np.zeros(sh + (4, 8))
    for mu in range(4):
        ax = AXIS[mu]
        umu = u[..., mu, :, :]
        xf = np.roll(x, -1, axis=ax)
        yf = np.roll(y, -1, axis=ax)
        v1 = np.einsum("st,...tc->...sc", ID4 - GAMMA[mu], np.einsum("...ab,...sb->...sa", umu, xf))
        q1 = np.einsum("...sa,...sb->...ab", v1, y.conj())
        v2 = np.einsum("...ab,...sb->...sa", umu, np.einsum("st,...tc->...sc", ID4 + GAMMA[mu], yf))
        q2 = np.einsum("...sa,...sb->...ab", x, v2.conj())
        bp = _bplus(dims, mu, bc)[..., None, None]
        q = bp * q1 - bp.conj() * q2
        g[..., mu, :] = -2.0 * kappa * np.einsum("aij,...ji->...a", T_GEN, q).imag
    return g.reshape(-1, 4, 8)


def fermion_action(U, phi, dims, kappa, mu, bc, tol: float = 1e-14, solve=None):
    """S_f = Re phi^dag (M^dag M)^{-1} phi.  Returns (S_f, X)."""
    if solve is None:
        x, _ = cg(lambda v: apply_MdagM(U, v, dims, kappa, mu, bc), phi, tol)
    else:
        x = solve(U, phi)
    return float(np.vdot(phi, x).real), x


def fermion_action_eo(U, phi_e, dims, kappa, mu, bc, tol: float = 1e-14):
    """S_f^eo = Re phi_e^dag (Mhat^dag Mhat)^{-1} phi_e.  Returns (S_f^eo, X_e)."""
    x, _ = cg(lambda v: apply_MhatdagMhat(U, v, dims, kappa, mu, bc), phi_e, tol)
    return float(np.vdot(phi_e, x).real), x


def fermion_force_eo(U, X_e, dims, kappa, mu, bc) -> np.ndarray:
    """dS_f^eo/dw^a for every link, shape (V, 4, 8), from X_e = (Mhat^dag Mhat)^{-1} phi_e."""
    y_e = apply_Mhat(U, X_e, dims, kappa, mu, bc)
    x_o = twist_inv(hop_pq(U, X_e, dims, bc, 1), kappa, mu)
    y_o = twist_inv(hop_pq(U, y_e, dims, bc, 1, dagger=True), kappa, -mu)
    x = to_full(X_e, dims, 0) + to_full(x_o, dims, 1)
    y = kappa * (to_full(y_e, dims, 0) + to_full(y_o, dims, 1))
    return fermion_force(U, x, y, dims, kappa, bc)


def _shift(a, dims, mu, step):
    """Field value at x + step*mu (periodic); a has lattice shape first."""
    return np.roll(a, -step, axis=AXIS[mu])


def plaquette_sum(U, dims) -> float:
    """sum_{x, mu<nu} Re Tr P_mu_nu(x), P = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag."""
    u = U.reshape(shape4(dims) + (4, 3, 3))
    total = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = u[..., mu, :, :] @ _shift(u[..., nu, :, :], dims, mu, 1)
            b = u[..., nu, :, :] @ _shift(u[..., mu, :, :], dims, nu, 1)
            total += float(np.sum(a * b.conj()).real)
    return float(total)


def gauge_action(U, dims, beta) -> float:
    n_plaq = 6 * int(np.prod(dims))
    return float(beta / 3.0 * (3.0 * n_plaq - plaquette_sum(U, dims)))


def staple_sum(U, dims) -> np.ndarray:
    """V_mu(x) such that the plaquettes holding U_mu(x) sum to Re Tr[U_mu(x) V_mu(x)]; (V, 4, 3, 3)."""
    sh = shape4(dims)
    u = U.reshape(sh + (4, 3, 3))
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    v = np.zeros_like(u)
    for mu in range(4):
        for nu in range(4):
            if nu == mu:
                continue
            u_nu_xmu = _shift(u[..., nu, :, :], dims, mu, 1)          # U_nu(x+mu)
            u_mu_xnu = _shift(u[..., mu, :, :], dims, nu, 1)          # U_mu(x+nu)
            v[..., mu, :, :] += u_nu_xmu @ dag(u_mu_xnu) @ dag(u[..., nu, :, :])
            u_nu_xmn = _shift(u_nu_xmu, dims, nu, -1)                  # U_nu(x+mu-nu)
            u_mu_xmn = _shift(u[..., mu, :, :], dims, nu, -1)          # U_mu(x-nu)
            u_nu_xmn2 = _shift(u[..., nu, :, :], dims, nu, -1)         # U_nu(x-nu)
            v[..., mu, :, :] += dag(u_nu_xmn) @ dag(u_mu_xmn) @ u_nu_xmn2
    return v.reshape(-1, 4, 3, 3)


def gauge_force(U, dims, beta) -> np.ndarray:
    """dS_g/dw^a, shape (V, 4, 8)."""
    uv = U @ staple_sum(U, dims)
    return beta / 3.0 * np.einsum("aij,...ji->...a", T_GEN, uv).imag
