"""FP64 oracle for the compressed link formats REC12, REC10 and REC8 (the paper's §4.1, Table 3).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.

For U in SU(3) with rows a, b, c (orthonormal, det U = 1):
* c = conj(a x b) (the paper's REC12: keep rows a and b, 12 reals);
* given the first row a and the first column (a1, b1, c1), the rest of b
  follows from two linear equations: a^dag-orthogonality of b,
      conj(a2) b2 + conj(a3) b3 = -conj(a1) b1,
  and the first component of c = conj(a x b),
      -a3 b2 + a2 b3 = conj(c1),
  whose determinant is |a2|^2 + |a3|^2; then c = conj(a x b).  REC10 stores
  a and (b1, c1): 10 reals.  (The paper only says that further restrictions on
  the 12 numbers save 2 or 4 more; this is the reading taken.)
* REC8 also drops |a1| and |c1|, which unitarity of the first row and of the
  first column gives back, |a1|^2 = 1 - |a2|^2 - |a3|^2 and |c1|^2 = 1 - |a1|^2
  - |b1|^2; it keeps their phases: 2 + 4 + 2 = 8 reals.
The system's determinant |a2|^2 + |a3|^2 vanishes when the first row is a pure
phase times (1, 0, 0): there the reconstruction loses accuracy as 1/(|a2|^2 +
|a3|^2), the arithmetic problem the paper mentions.
"""
from __future__ import annotations

import numpy as np

__all__ = ["rec12_decode", "rec10_encode", "rec10_decode", "rec8_encode", "rec8_decode"]


def rec12_decode(ab):
    """Links from their first two rows ab[..., 2, 3]."""
    a, b = ab[..., 0, :], ab[..., 1, :]
    return np.stack([a, b, np.conj(np.cross(a, b))], axis=-2)


def rec10_encode(U):
    """(a[..., 3], b1[...], c1[...]): the first row and the rest of the first column."""
    return U[..., 0, :].copy(), U[..., 1, 0].copy(), U[..., 2, 0].copy()


def _complete(a, b1, c1):
    """The link with first row a and first column (a1, b1, c1)."""
    m = np.empty(a.shape[:-1] + (2, 2), dtype=np.complex128)
    m[..., 0, 0], m[..., 0, 1] = np.conj(a[..., 1]), np.conj(a[..., 2])
    m[..., 1, 0], m[..., 1, 1] = -a[..., 2], a[..., 1]
    rhs = np.stack([-np.conj(a[..., 0]) * b1, np.conj(c1)], axis=-1)
    b23 = np.linalg.solve(m, rhs[..., None])[..., 0]
    b = np.concatenate([b1[..., None], b23], axis=-1)
    return rec12_decode(np.stack([a, b], axis=-2))


def rec10_decode(enc):
    a, b1, c1 = enc
    return _complete(a, b1, c1)


def rec8_encode(U):
    """(theta_a, theta_c, a2, a3, b1): the phases of a1 and c1 and three complex entries."""
    return np.angle(U[..., 0, 0]), np.angle(U[..., 2, 0]), U[..., 0, 1].copy(), U[..., 0, 2].copy(), U[..., 1, 0].copy()


def rec8_decode(enc):
    th_a, th_c, a2, a3, b1 = enc
    a1 = np.sqrt(np.maximum(0.0, 1.0 - np.abs(a2) ** 2 - np.abs(a3) ** 2)) * np.exp(1j * th_a)
    c1 = np.sqrt(np.maximum(0.0, 1.0 - np.abs(a1) ** 2 - np.abs(b1) ** 2)) * np.exp(1j * th_c)
    return _complete(np.stack([a1, a2, a3], axis=-1), b1, c1)
