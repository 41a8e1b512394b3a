"""Seeded synthetic inputs for the twisted-mass Wilson operator.

This module only *draws* inputs; it holds none of the operator, solver or
force arithmetic.  Both the GPU path and the FP64 oracle read the bytes it
produces, so a parity test compares the two on identical fields.

Canonical host layouts (complex128, site index s = x + Lx*(y + Ly*(z + Lz*t)),
x fastest; direction mu = 0,1,2,3 <-> x,y,z,t):

* gauge field  U[s, mu, a, b]       shape (V, 4, 3, 3)
  -- U_mu(s) is the link from s to s + mu_hat (paper, section 2.1)
* spinor       psi[s, spin, colour] shape (V, 4, 3)
* momenta      p[s, mu, a]          shape (V, 4, 8) real, coefficient of T^a

The paper's production runs start from thermalised configurations; none are
available, so links are drawn as U = exp(i*eps*sum_a c_a lambda_a) with
c_a ~ N(0, 1): unitary, unit determinant, with disorder set by eps.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "gell_mann", "random_links", "unit_links", "gaussian_spinor",
    "point_sources", "random_gauge_transform", "gaussian_momenta",
    "random_link_sample",
]


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda^a, shape (8, 3, 3), hermitian and traceless."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _su3_from_coefficients(c: np.ndarray, eps: float, chunk: int = 1 << 20) -> np.ndarray:
    """exp(i*eps*sum_a c[..., a] lambda^a) for real c of shape (..., 8), via eigh."""
    lam = gell_mann()
    flat = c.reshape(-1, 8)
    out = np.empty((flat.shape[0], 3, 3), dtype=np.complex128)
    for i0 in range(0, flat.shape[0], chunk):
        h = np.einsum("na,aij->nij", flat[i0:i0 + chunk], lam)
        w, v = np.linalg.eigh(h)
        out[i0:i0 + chunk] = np.einsum("nij,nj,nkj->nik", v, np.exp(1j * eps * w), v.conj())
    return out.reshape(c.shape[:-1] + (3, 3))


def random_links(dims, eps: float, seed: int) -> np.ndarray:
    """Gauge field of shape (V, 4, 3, 3): U = exp(i eps sum_a c_a lambda_a), c ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(volume(dims), 4, 8))
    return _su3_from_coefficients(c, eps)


def unit_links(dims) -> np.ndarray:
    """The free field U = 1, shape (V, 4, 3, 3)."""
    u = np.zeros((volume(dims), 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def gaussian_spinor(n_sites: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian spinor, re and im ~ N(0, 1/2): shape (n_sites, 4, 3) or (nrhs, n_sites, 4, 3)."""
    rng = np.random.default_rng(seed)
    shape = (n_sites, 4, 3) if nrhs is None else (nrhs, n_sites, 4, 3)
    re = rng.normal(size=shape)
    im = rng.normal(size=shape)
    return (re + 1j * im) * np.sqrt(0.5)


def point_sources(n_sites: int, site: int = 0) -> np.ndarray:
    """The 12 spin-colour point sources at one site: shape (12, n_sites, 4, 3).

    Column k = 3*spin + colour holds delta_{x,site} delta_{s,spin} delta_{c,colour}.
    """
    b = np.zeros((12, n_sites, 4, 3), dtype=np.complex128)
    for k in range(12):
        b[k, site, k // 3, k % 3] = 1
    return b


def random_gauge_transform(n_sites: int, eps: float, seed: int) -> np.ndarray:
    """One random SU(3) matrix per site, shape (n_sites, 3, 3)."""
    rng = np.random.default_rng(seed)
    return _su3_from_coefficients(rng.normal(size=(n_sites, 8)), eps)


def gaussian_momenta(n_sites: int, seed: int) -> np.ndarray:
    """HMC momenta p^a ~ N(0, 1), shape (n_sites, 4, 8), float64."""
    return np.random.default_rng(seed).normal(size=(n_sites, 4, 8))


def random_link_sample(n_sites: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct random links (site, mu), shape (count, 2), int64."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(n_sites * 4, size=count, replace=False)
    return np.stack([flat // 4, flat % 4], axis=1).astype(np.int64)
