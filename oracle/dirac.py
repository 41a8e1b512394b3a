"""FP64 oracle for the twisted-mass Wilson operator and its even-odd Schur complement.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.  It shares no code with the HIP path.

Definitions follow the paper's fermion-matrix section (the equation defining
D_tm^{+-} = M_diag^{+-} + Dslash, and the text after it):

* M = D_tm^+ = A - kappa*H, A = 1 + i*w*gamma5, w = 2*kappa*mu.  The paper prints
  the hopping prefactor as kappa/2; we read it as kappa, which makes the free
  massless operator at kappa = 1/8 massless as the paper's kappa = 1/(2(am+4))
  requires.
* (H psi)(x) = sum_mu [ b+_mu(x) (1 - gamma_mu) U_mu(x) psi(x+mu)
                       + b-_mu(x) (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ],
  i.e. the paper's sum over +-mu with gamma_{-mu} = -gamma_mu and
  U_{-mu}(x) = U_mu(x-mu)^dag.  b+_mu(x) = bc_mu when x_mu = L_mu - 1, else 1;
  b-_mu(x) = conj(bc_mu) when x_mu = 0, else 1 (phase only on boundary hops).
* Even-odd preconditioning (paper, section 2.1 on solvers): the Schur complement
  on even sites Mhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe.

Gamma matrices: the paper fixes only {gamma_mu, gamma_nu} = 2 delta.  We use the
Euclidean chiral basis gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = x,y,z),
gamma_t = [[0, -1], [-1, 0]], gamma5 = gamma_x gamma_y gamma_z gamma_t
= diag(-1, -1, 1, 1).

Site order: s = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) mod 2; the half
field of one parity is indexed by h = s >> 1.  Fields are complex128 arrays
psi[V, 4, 3] and U[V, 4, 3, 3].
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "GAMMA", "GAMMA5", "ID4", "shape4", "AXIS", "coords", "site_parity", "half_sites",
    "to_half", "to_full", "hop", "hop_pq", "twist", "twist_inv", "gamma5", "apply_M",
    "apply_Mdag", "apply_MdagM", "apply_Mhat", "apply_Mhatdag", "apply_MhatdagMhat",
    "apply_op", "dense_matrix", "cg", "solve_eo", "true_rel_residual", "hop_at_sites",
    "OPS",
]

_SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)


def _gammas() -> np.ndarray:
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    for k in range(3):
        g[k, :2, 2:] = -1j * _SIGMA[k]
        g[k, 2:, :2] = 1j * _SIGMA[k]
    g[3, :2, 2:] = -np.eye(2)
    g[3, 2:, :2] = -np.eye(2)
    return g


GAMMA = _gammas()
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)

# direction mu -> numpy axis of the (Lt, Lz, Ly, Lx) view
AXIS = (3, 2, 1, 0)


def shape4(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def coords(dims) -> np.ndarray:
    """Coordinates (x, y, z, t) of every site in lexicographic order, shape (V, 4)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    s = np.arange(lx * ly * lz * lt)
    return np.stack([s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)], axis=1)


def site_parity(dims) -> np.ndarray:
    return coords(dims).sum(axis=1) % 2


def half_sites(dims, parity: int) -> np.ndarray:
    """Sites of one parity in the order of their half index h = s >> 1."""
    s = np.nonzero(site_parity(dims) == parity)[0]
    assert np.array_equal(s >> 1, np.arange(s.size)), "half index must be s >> 1 (Lx even)"
    return s


def to_half(full: np.ndarray, dims, parity: int) -> np.ndarray:
    """Restrict a full field (..., V, 4, 3) to the sites of one parity."""
    return full[..., half_sites(dims, parity), :, :]


def to_full(half: np.ndarray, dims, parity: int) -> np.ndarray:
    """Embed a half field into the full lattice, zero on the other parity."""
    v = int(np.prod(dims))
    out = np.zeros(half.shape[:-3] + (v, 4, 3), dtype=np.complex128)
    out[..., half_sites(dims, parity), :, :] = half
    return out


def _scale_slice(a: np.ndarray, axis: int, index: int, factor: complex) -> None:
    if factor == 1:
        return
    sl = [slice(None)] * a.ndim
    sl[axis] = index
    a[tuple(sl)] *= factor


def hop(U, psi, dims, bc, dagger: bool = False) -> np.ndarray:
    """Hopping term H psi (dagger=False) or its conjugate transpose H^dag psi.

    H^dag is H with gamma_mu -> -gamma_mu: the adjoint of the forward term at x
    is a backward term at x + mu with the projector (1 - gamma_mu) and the
    conjugate phase, and vice versa.
    """
    sgn = -1.0 if dagger else 1.0
    nb_dims = psi.ndim - 3                     # leading batch dimensions, if any
    f = psi.reshape(psi.shape[:-3] + shape4(dims) + (4, 3))
    u = U.reshape(shape4(dims) + (4, 3, 3))
    out = np.zeros_like(f)
    for mu in range(4):
        ax, length = nb_dims + AXIS[mu], int(dims[mu])
        umu = u[..., mu, :, :]
        # forward: b+(x) (1 - s gamma_mu) U_mu(x) psi(x + mu)
        nb = np.roll(f, -1, axis=ax)
        _scale_slice(nb, ax, length - 1, complex(bc[mu]))
        t = np.einsum("...ab,...sb->...sa", umu, nb)
        out += np.einsum("st,...tc->...sc", ID4 - sgn * GAMMA[mu], t)
        # backward: b-(x) (1 + s gamma_mu) U_mu(x - mu)^dag psi(x - mu)
        w = np.einsum("...ba,...sb->...sa", umu.conj(), f)
        nb = np.roll(w, 1, axis=ax)
        _scale_slice(nb, ax, 0, np.conj(complex(bc[mu])))
        out += np.einsum("st,...tc->...sc", ID4 + sgn * GAMMA[mu], nb)
    return out.reshape(psi.shape)


def hop_pq(U, psi_q, dims, bc, out_parity: int, dagger: bool = False) -> np.ndarray:
    """H_pq: the hop restricted to parity-q input and parity-p output (q = 1 - p)."""
    full = to_full(psi_q, dims, 1 - out_parity)
    return to_half(hop(U, full, dims, bc, dagger), dims, out_parity)


def gamma5(psi) -> np.ndarray:
    return np.einsum("st,...tc->...sc", GAMMA5, psi)


def twist(psi, kappa, mu) -> np.ndarray:
    """A psi = (1 + i 2 kappa mu gamma5) psi."""
    a = ID4 + 2j * kappa * mu * GAMMA5
    return np.einsum("st,...tc->...sc", a, psi)


def twist_inv(psi, kappa, mu) -> np.ndarray:
    """A^{-1} psi, with A^{-1} the inverse of the 4x4 spin matrix of A."""
    a_inv = np.linalg.inv(ID4 + 2j * kappa * mu * GAMMA5)
    return np.einsum("st,...tc->...sc", a_inv, psi)


def apply_M(U, psi, dims, kappa, mu, bc) -> np.ndarray:
    return twist(psi, kappa, mu) - kappa * hop(U, psi, dims, bc)


def apply_Mdag(U, psi, dims, kappa, mu, bc) -> np.ndarray:
    """M^dag = A^dag - kappa H^dag, with A^dag = 1 - i w gamma5."""
    return twist(psi, kappa, -mu) - kappa * hop(U, psi, dims, bc, dagger=True)


def apply_MdagM(U, psi, dims, kappa, mu, bc) -> np.ndarray:
    return apply_Mdag(U, apply_M(U, psi, dims, kappa, mu, bc), dims, kappa, mu, bc)


def apply_Mhat(U, psi_e, dims, kappa, mu, bc) -> np.ndarray:
    """Mhat psi_e = A_ee psi_e - kappa^2 H_eo A_oo^{-1} H_oe psi_e."""
    t = twist_inv(hop_pq(U, psi_e, dims, bc, 1), kappa, mu)
    return twist(psi_e, kappa, mu) - kappa ** 2 * hop_pq(U, t, dims, bc, 0)


def apply_Mhatdag(U, psi_e, dims, kappa, mu, bc) -> np.ndarray:
    """Mhat^dag = A^dag - kappa^2 (H_oe)^dag A^{-dag} (H_eo)^dag.

    (H_oe)^dag = (P_o H P_e)^dag = P_e H^dag P_o, the even-output part of H^dag.
    """
    t = twist_inv(hop_pq(U, psi_e, dims, bc, 1, dagger=True), kappa, -mu)
    return twist(psi_e, kappa, -mu) - kappa ** 2 * hop_pq(U, t, dims, bc, 0, dagger=True)


def apply_MhatdagMhat(U, psi_e, dims, kappa, mu, bc) -> np.ndarray:
    return apply_Mhatdag(U, apply_Mhat(U, psi_e, dims, kappa, mu, bc), dims, kappa, mu, bc)


def _dslash_eo(U, psi, dims, kappa, mu, bc):
    return -kappa * hop_pq(U, psi, dims, bc, 0)


def _dslash_oe(U, psi, dims, kappa, mu, bc):
    return -kappa * hop_pq(U, psi, dims, bc, 1)


# Operator names shared with the C interface; each maps to its definition above.
OPS = {
    "DSLASH_EO": _dslash_eo,
    "DSLASH_OE": _dslash_oe,
    "M": apply_M,
    "MDAG": apply_Mdag,
    "MDAGM": apply_MdagM,
    "MHAT": apply_Mhat,
    "MHATDAG": apply_Mhatdag,
    "MHATDAGMHAT": apply_MhatdagMhat,
}


def apply_op(name, U, psi, dims, kappa, mu, bc):
    return OPS[name](U, psi, dims, kappa, mu, bc)


def dense_matrix(apply, n_sites: int, chunk: int = 192) -> np.ndarray:
    """Dense matrix of a linear map on (n_sites, 4, 3) fields, by applying it to unit vectors.

    `apply` must accept a leading batch dimension; columns are formed in chunks.
    """
    n = 12 * n_sites
    m = np.empty((n, n), dtype=np.complex128)
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        e = np.zeros((j1 - j0, n), dtype=np.complex128)
        e[np.arange(j1 - j0), np.arange(j0, j1)] = 1
        m[:, j0:j1] = apply(e.reshape(j1 - j0, n_sites, 4, 3)).reshape(j1 - j0, n).T
    return m


def cg(apply_A, b, tol: float = 1e-10, maxiter: int = 100000, x0=None):
    """Hestenes-Stiefel CG for a hermitian positive-definite map; stops on ||r||/||b|| <= tol.

    Returns (x, iterations).  r is the recursively updated residual.
    """
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128, copy=True)
    r = b - apply_A(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    bb = np.vdot(b, b).real
    k = 0
    while k < maxiter and rr > tol * tol * bb:
        ap = apply_A(p)
        alpha = rr / np.vdot(p, ap).real
        x += alpha * p
        r -= alpha * ap
        rr_new = np.vdot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
    return x, k


def true_rel_residual(apply_A, b, x) -> float:
    """||b - A x||_2 / ||b||_2, recomputed in FP64."""
    return float(np.linalg.norm(b - apply_A(x)) / np.linalg.norm(b))


def solve_eo(U, b, dims, kappa, mu, bc, tol: float = 1e-13):
    """Solve M x = b through the even-site Schur complement.

    x_e = Mhat^{-1}(b_e + kappa H_eo A^{-1} b_o), x_o = A^{-1}(b_o + kappa H_oe x_e);
    Mhat^{-1} is applied as Mhat^{-1} = (Mhat^dag Mhat)^{-1} Mhat^dag with CG.
    """
    be, bo = to_half(b, dims, 0), to_half(b, dims, 1)
    rhs = be + kappa * hop_pq(U, twist_inv(bo, kappa, mu), dims, bc, 0)
    normal_rhs = apply_Mhatdag(U, rhs, dims, kappa, mu, bc)
    xe, _ = cg(lambda v: apply_MhatdagMhat(U, v, dims, kappa, mu, bc), normal_rhs, tol)
    xo = twist_inv(bo + kappa * hop_pq(U, xe, dims, bc, 1), kappa, mu)
    return to_full(xe, dims, 0) + to_full(xo, dims, 1)


def hop_at_sites(U, psi, dims, bc, sites, dagger: bool = False) -> np.ndarray:
    """(H psi)(x) at the listed full-lattice sites only, term by term.

    For sampled checks on lattices where the whole-lattice hop is not wanted.
    Returns shape (len(sites), 4, 3).
    """
    sgn = -1.0 if dagger else 1.0
    lx, ly, lz, lt = (int(d) for d in dims)
    ext = (lx, ly, lz, lt)
    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for i, s in enumerate(sites):
        s = int(s)
        c = [s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)]
        for mu in range(4):
            cf, cb = list(c), list(c)
            cf[mu] = (c[mu] + 1) % ext[mu]
            cb[mu] = (c[mu] - 1) % ext[mu]
            sf = cf[0] + lx * (cf[1] + ly * (cf[2] + lz * cf[3]))
            sb = cb[0] + lx * (cb[1] + ly * (cb[2] + lz * cb[3]))
            bf = complex(bc[mu]) if c[mu] == ext[mu] - 1 else 1.0
            bb = np.conj(complex(bc[mu])) if c[mu] == 0 else 1.0
            fwd = bf * (ID4 - sgn * GAMMA[mu]) @ (psi[sf] @ U[s, mu].T)
            bwd = bb * (ID4 + sgn * GAMMA[mu]) @ (psi[sb] @ U[sb, mu].conj())
            out[i] += fwd + bwd
    return out
