"""ctypes front end of the plain C++/OpenMP FP64 oracle (oracle/cpu/tmqcd_ref.cpp).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.  The C++ oracle follows the same
definitions as oracle/dirac.py (the paper's D_tm equation and its even-odd
Schur complement, section 2.1) in loops over sites, so that the operator, the
Schur complement and CG run at full lattice sizes on the host cores; it is
pinned against the NumPy oracle and the free-field closed form by
tests/test_oracle_cref.py.

build() compiles it with g++ (-O2, OpenMP, no target-specific flags: the
baseline as written, not tuned for a host).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu", "tmqcd_ref.cpp")
LIB = os.path.join(HERE, "cpu", "libtmqcd_ref.so")

OPS = {"H": 0, "M": 1, "MDAG": 2, "MDAGM": 3, "MHAT": 4, "MHATDAG": 5, "MHATDAGMHAT": 6, "HOP_EO": 7, "HOP_OE": 8}
FULL_OPS = ("H", "M", "MDAG", "MDAGM")

_lib = None


def build() -> str:
    """Compile the C++ oracle into oracle/cpu/libtmqcd_ref.so (always); returns its path."""
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O2", "-fcx-limited-range", "-fopenmp", "-fPIC", "-shared", "-std=c++17", SRC, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"g++ failed on {SRC}:\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        I, D, P, DP = ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p
        L.ref_threads.restype, L.ref_threads.argtypes = I, []
        L.ref_set_threads.restype, L.ref_set_threads.argtypes = None, [I]
        L.ref_apply.restype, L.ref_apply.argtypes = I, [I, P, D, D, DP, DP, DP, DP]
        L.ref_true_rel_residual.restype = D
        L.ref_true_rel_residual.argtypes = [I, P, D, D, DP, DP, DP, DP]
        L.ref_cg.restype, L.ref_cg.argtypes = I, [I, P, D, D, DP, DP, DP, DP, D, I, D, DP]
        _lib = L
    return _lib


def threads() -> int:
    return lib().ref_threads()


def set_threads(n: int) -> None:
    lib().ref_set_threads(int(n))


def _args(dims, bc):
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    b = np.array([[complex(v).real, complex(v).imag] for v in bc], dtype=np.float64)
    return d, b


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check_shapes(op: str, U, psi, dims):
    """The C++ side trusts the sizes: check them here (links (V, 4, 3, 3); fields (n, 4, 3))."""
    v = int(np.prod([int(d) for d in dims]))
    n = v if op in FULL_OPS else v // 2
    if U.size != v * 36 or psi.size != n * 12:
        raise ValueError(f"{op}: links of {U.size // 36} sites and a field of {psi.size // 12} sites for extents "
                         f"{tuple(dims)} (want {v} and {n})")


def apply(op: str, U, psi, dims, kappa, mu, bc) -> np.ndarray:
    """op(psi) for op in OPS; psi (V, 4, 3) for the full-lattice ops, (V/2, 4, 3) otherwise."""
    d, b = _args(dims, bc)
    U, psi = _c128(U), _c128(psi)
    _check_shapes(op, U, psi, dims)
    out = np.empty_like(psi)
    rc = lib().ref_apply(OPS[op], d, float(kappa), float(mu), _p(b), _p(U), _p(psi), _p(out))
    if rc != 0:
        raise ValueError(f"ref_apply({op}) failed: {rc}")
    return out


def true_rel_residual(op: str, U, b, x, dims, kappa, mu, bc) -> float:
    """||b - op x|| / ||b|| in FP64."""
    d, bcv = _args(dims, bc)
    U, b, x = _c128(U), _c128(b), _c128(x)
    _check_shapes(op, U, b, dims)
    _check_shapes(op, U, x, dims)
    return lib().ref_true_rel_residual(OPS[op], d, float(kappa), float(mu), _p(bcv), _p(U), _p(b), _p(x))


def cg(op: str, U, b, dims, kappa, mu, bc, tol=1e-10, max_iter=100000, report_tol=None):
    """CG on MDAGM or MHATDAGMHAT from x = 0.  Returns (x, stats dict, return code)."""
    d, bcv = _args(dims, bc)
    U, b = _c128(U), _c128(b)
    _check_shapes(op, U, b, dims)
    x = np.empty_like(b)
    st = np.zeros(6)
    rc = lib().ref_cg(OPS[op], d, float(kappa), float(mu), _p(bcv), _p(U), _p(b), _p(x), float(tol), int(max_iter),
                      float(report_tol if report_tol is not None else tol), _p(st))
    if rc < 0:
        raise ValueError(f"ref_cg failed: {rc}")
    return x, {"iters": int(st[0]), "true_rel_residual": float(st[1]), "seconds": float(st[2]),
               "report_iters": int(st[3]), "report_seconds": float(st[4]),
               "report_true_rel_residual": float(st[5])}, rc
