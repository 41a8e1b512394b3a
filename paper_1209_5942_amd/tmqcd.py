"""Thin ctypes binding of libtmqcd.so (the C interface in include/tmqcd.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device memory comes from torch (``torch.empty(..., device="cuda")``)
and calls are ordered on ``torch.cuda.current_stream()`` unless a stream is
given.  The library must be built (``python -m paper_1209_5942_amd.build``);
loading raises ``TmqcdLibraryMissing`` otherwise - there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtmqcd.so")

# constants of include/tmqcd.h
OK, EINVAL, EALIAS, EALIGN, ENOCONV, EBREAKDOWN, EHIP, EWORKSPACE, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7, -8
F64, F32, F16 = 0, 1, 2
RECON18, RECON12, RECON10, RECON8 = 0, 1, 2, 3
FULL, EVEN, ODD = 0, 1, 2
DSLASH_EO, DSLASH_OE, M, MDAG, MDAGM, MHAT, MHATDAG, MHATDAGMHAT = range(8)
OPS = {"DSLASH_EO": DSLASH_EO, "DSLASH_OE": DSLASH_OE, "M": M, "MDAG": MDAG, "MDAGM": MDAGM,
       "MHAT": MHAT, "MHATDAG": MHATDAG, "MHATDAGMHAT": MHATDAGMHAT}
OP_SUBSETS = {DSLASH_EO: (ODD, EVEN), DSLASH_OE: (EVEN, ODD), M: (FULL, FULL), MDAG: (FULL, FULL),
              MDAGM: (FULL, FULL), MHAT: (EVEN, EVEN), MHATDAG: (EVEN, EVEN), MHATDAGMHAT: (EVEN, EVEN)}

ENTRY_POINTS = ("tmqcd_gauge_bytes", "tmqcd_spinor_bytes", "tmqcd_workspace_bytes", "tmqcd_pack_gauge",
                "tmqcd_unpack_gauge", "tmqcd_pack_spinor", "tmqcd_unpack_spinor", "tmqcd_dslash", "tmqcd_cg",
                "tmqcd_cg_batch_workspace_bytes", "tmqcd_cg_batch", "tmqcd_bicgstab_workspace_bytes",
                "tmqcd_bicgstab", "tmqcd_force_workspace_bytes", "tmqcd_force", "tmqcd_force_eo_workspace_bytes", "tmqcd_force_eo",
                "tmqcd_gauge_force", "tmqcd_gauge_force_tlsym_workspace_bytes", "tmqcd_gauge_force_tlsym", "tmqcd_rectangle", "tmqcd_heatbath",
                "tmqcd_overrelax", "tmqcd_update_links", "tmqcd_tune_workspace_bytes", "tmqcd_tune",
                "tmqcd_tune_save", "tmqcd_tune_load", "tmqcd_tune_clear", "tmqcd_tune_set",
                "tmqcd_tune_mrhs_workspace_bytes", "tmqcd_tune_mrhs", "tmqcd_plaquette", "tmqcd_momentum_norm2",
                "tmqcd_dot", "tmqcd_delta_h", "tmqcd_hbm_probe", "tmqcd_error_string", "tmqcd_last_hip_error",
                "tmqcd_noalloc_scratch_bytes", "tmqcd_dslash_noalloc")


class TmqcdLibraryMissing(RuntimeError):
    pass


class TmqcdError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {error_string(code)} (code {code}, hip error {last_hip_error()})")


class CProblem(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("kappa", ctypes.c_double), ("mu", ctypes.c_double),
                ("bc", (ctypes.c_double * 2) * 4)]


class CCgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("op", ctypes.c_int32),
                ("inner_prec", ctypes.c_int32), ("recon", ctypes.c_int32), ("reliable_delta", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("x_is_zero", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("nrhs", ctypes.c_int32)]


class CCgStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("reliable_updates", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("hop_launches", ctypes.c_int32), ("true_rel_residual", ctypes.c_double),
                ("iter_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("inner_iters", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class CTuneResult(ctypes.Structure):
    _fields_ = [("kernel_class", ctypes.c_int32), ("block", ctypes.c_int32), ("order", ctypes.c_int32),
                ("group", ctypes.c_int32), ("candidates", ctypes.c_int32), ("rejected", ctypes.c_int32),
                ("us", ctypes.c_double), ("default_us", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libtmqcd.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TmqcdLibraryMissing(f"{LIB_PATH} is missing: run `python -m paper_1209_5942_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, V, I, S, D = ctypes.POINTER(CProblem), ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
        sig = {
            "tmqcd_gauge_bytes": (S, [P, I, I]),
            "tmqcd_spinor_bytes": (S, [P, I, I, I]),
            "tmqcd_workspace_bytes": (S, [P, I, I, I]),
            "tmqcd_pack_gauge": (I, [P, V, V, I, I, V]),
            "tmqcd_unpack_gauge": (I, [P, V, V, I, I, V]),
            "tmqcd_pack_spinor": (I, [P, V, V, I, I, I, V]),
            "tmqcd_unpack_spinor": (I, [P, V, V, I, I, I, V]),
            "tmqcd_dslash": (I, [P, V, V, V, I, I, I, I, V, S, V]),
            "tmqcd_cg": (I, [P, ctypes.POINTER(V * 3), V, V, ctypes.POINTER(CCgOpts), ctypes.POINTER(CCgStats),
                             V, S, V]),
            "tmqcd_cg_batch_workspace_bytes": (S, [I, P]),
            "tmqcd_bicgstab_workspace_bytes": (S, [P, I]),
            "tmqcd_bicgstab": (I, [P, V, V, V, ctypes.POINTER(CCgOpts), ctypes.POINTER(CCgStats), V, S, V]),
            "tmqcd_cg_batch": (I, [I, P, V, V, V, ctypes.POINTER(CCgOpts), ctypes.POINTER(CCgStats), I, V, S, V]),
            "tmqcd_force_workspace_bytes": (S, [P]),
            "tmqcd_force": (I, [P, V, I, V, V, V, D, I, V, S, V]),
            "tmqcd_force_eo_workspace_bytes": (S, [P]),
            "tmqcd_force_eo": (I, [P, V, I, V, V, D, I, V, S, V]),
            "tmqcd_gauge_force": (I, [P, V, D, V, D, I, V]),
            "tmqcd_gauge_force_tlsym_workspace_bytes": (S, [P]),
            "tmqcd_gauge_force_tlsym": (I, [P, V, D, D, V, D, I, V, S, V]),
            "tmqcd_rectangle": (I, [P, V, V, V, S, V]),
            "tmqcd_heatbath": (I, [P, V, I, D, ctypes.c_uint64, ctypes.c_uint32, V]),
            "tmqcd_overrelax": (I, [P, V, I, V]),
            "tmqcd_update_links": (I, [P, V, V, D, V]),
            "tmqcd_plaquette": (I, [P, V, V, V, S, V]),
            "tmqcd_momentum_norm2": (I, [P, V, V, V, S, V]),
            "tmqcd_dot": (I, [P, V, V, I, V, V, S, V]),
            "tmqcd_delta_h": (I, [P, V, V, V, V, V, V, V, I, D, D, V, V, S, V]),
            "tmqcd_tune_workspace_bytes": (S, [P, I]),
            "tmqcd_tune": (I, [P, V, I, I, V, S, ctypes.POINTER(CTuneResult), V]),
            "tmqcd_tune_save": (I, [ctypes.c_char_p]),
            "tmqcd_tune_load": (I, [ctypes.c_char_p]),
            "tmqcd_tune_clear": (None, []),
            "tmqcd_tune_set": (I, [P, I, I, I, I, I, I, I]),
            "tmqcd_tune_mrhs_workspace_bytes": (S, [P, I, I]),
            "tmqcd_tune_mrhs": (I, [P, V, I, I, I, V, S, ctypes.POINTER(CTuneResult), V]),
            "tmqcd_hbm_probe": (I, [V, V, S, I, V, V]),
            "tmqcd_error_string": (ctypes.c_char_p, [I]),
            "tmqcd_last_hip_error": (I, []),
            "tmqcd_noalloc_scratch_bytes": (S, []),
            "tmqcd_dslash_noalloc": (I, [P, V, V, V, I, I, I, I, V]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().tmqcd_error_string(code).decode()


def last_hip_error() -> int:
    return lib().tmqcd_last_hip_error()


def _check(code: int, where: str):
    if code != OK:
        raise TmqcdError(code, where)


@dataclass
class Problem:
    """Lattice extents (Lx, Ly, Lz, Lt), kappa, mu and per-direction boundary phases."""
    dims: tuple
    kappa: float
    mu: float
    bc: tuple = (1, 1, 1, -1)

    def c(self) -> CProblem:
        p = CProblem()
        for i in range(4):
            p.dims[i] = int(self.dims[i])
            z = complex(self.bc[i])
            p.bc[i][0], p.bc[i][1] = z.real, z.imag
        p.kappa, p.mu = float(self.kappa), float(self.mu)
        return p

    @property
    def volume(self) -> int:
        v = 1
        for d in self.dims:
            v *= int(d)
        return v


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _bytes(n: int, device="cuda"):
    import torch
    return torch.empty(int(n), dtype=torch.uint8, device=device)


def gauge_bytes(prob: Problem, prec=F64, recon=RECON18) -> int:
    return lib().tmqcd_gauge_bytes(ctypes.byref(prob.c()), prec, recon)


def spinor_bytes(prob: Problem, prec=F64, subset=FULL, nrhs=1) -> int:
    return lib().tmqcd_spinor_bytes(ctypes.byref(prob.c()), prec, subset, nrhs)


def workspace_bytes(prob: Problem, op: int, prec_mask: int = 1, nrhs: int = 1) -> int:
    return lib().tmqcd_workspace_bytes(ctypes.byref(prob.c()), op, prec_mask, nrhs)


def workspace(prob: Problem, op: int, prec_mask: int = 1 | 2 | 4, nrhs: int = 1):
    return _bytes(workspace_bytes(prob, op, prec_mask, nrhs))


def pack_gauge(prob: Problem, U_canon, prec=F64, recon=RECON18, out=None, stream=None):
    """U_canon: complex128 device tensor (V, 4, 3, 3) -> packed uint8 device tensor."""
    assert U_canon.is_contiguous()
    out = _bytes(gauge_bytes(prob, prec, recon)) if out is None else out
    _check(lib().tmqcd_pack_gauge(ctypes.byref(prob.c()), _ptr(U_canon), _ptr(out), prec, recon, _stream(stream)),
           "tmqcd_pack_gauge")
    return out


def unpack_gauge(prob: Problem, U_packed, prec=F64, recon=RECON18, stream=None):
    """Packed links -> complex128 device tensor (V, 4, 3, 3)."""
    import torch
    out = torch.empty((prob.volume, 4, 3, 3), dtype=torch.complex128, device=U_packed.device)
    _check(lib().tmqcd_unpack_gauge(ctypes.byref(prob.c()), _ptr(U_packed), _ptr(out), prec, recon, _stream(stream)),
           "tmqcd_unpack_gauge")
    return out


def pack_spinor(prob: Problem, psi, prec=F64, subset=FULL, nrhs=1, out=None, stream=None):
    """psi: complex128 device tensor ([nrhs,] n, 4, 3) -> packed uint8 device tensor."""
    assert psi.is_contiguous()
    out = _bytes(spinor_bytes(prob, prec, subset, nrhs)) if out is None else out
    _check(lib().tmqcd_pack_spinor(ctypes.byref(prob.c()), _ptr(psi), _ptr(out), prec, subset, nrhs,
                                   _stream(stream)), "tmqcd_pack_spinor")
    return out


def unpack_spinor(prob: Problem, packed, prec=F64, subset=FULL, nrhs=1, stream=None):
    import torch
    n = prob.volume if subset == FULL else prob.volume // 2
    shape = (n, 4, 3) if nrhs == 1 else (nrhs, n, 4, 3)
    out = torch.empty(shape, dtype=torch.complex128, device=packed.device)
    _check(lib().tmqcd_unpack_spinor(ctypes.byref(prob.c()), _ptr(packed), _ptr(out), prec, subset, nrhs,
                                     _stream(stream)), "tmqcd_unpack_spinor")
    return out


def dslash(prob: Problem, U_packed, inp, op, prec=F64, recon=RECON18, nrhs=1, ws=None, out=None, stream=None):
    """out = op(inp) on packed fields."""
    if out is None:
        out = _bytes(spinor_bytes(prob, prec, OP_SUBSETS[op][1], nrhs))
    if ws is None:
        ws = _bytes(workspace_bytes(prob, op, 1 << prec, nrhs))
    _check(lib().tmqcd_dslash(ctypes.byref(prob.c()), _ptr(U_packed), _ptr(inp), _ptr(out), op, prec, recon, nrhs,
                              _ptr(ws), ws.numel(), _stream(stream)), "tmqcd_dslash")
    return out


def dslash_noalloc(prob: Problem, U_packed, inp, out, op, prec=F64, recon=RECON18, nrhs=1, stream=None):
    """out = op(inp) on packed fields, the temporaries in the library's static scratch (no allocation
    by the library; `out` is the caller's)."""
    _check(lib().tmqcd_dslash_noalloc(ctypes.byref(prob.c()), _ptr(U_packed), _ptr(inp), _ptr(out), op, prec, recon,
                                      nrhs, _stream(stream)), "tmqcd_dslash_noalloc")
    return out


def cg(prob: Problem, U_packed: dict, b, x=None, *, x_is_zero=None, tol=1e-10, max_iter=10000, op=MHATDAGMHAT,
       inner_prec=F64, recon=RECON18, reliable_delta=0.0, check_every=0, ws=None, stream=None,
       raise_on_noconv=True, use_graph=0, nrhs=1, raise_on_breakdown=True):
    """Solve op x = b (packed FP64 fields).  U_packed maps precision -> packed gauge field.

    x: output buffer (allocated when None).  x_is_zero: start from x0 = 0 (default: when x is None);
    otherwise the contents of x are the start vector.  use_graph: 1 replays the iterations from a
    captured hipGraph, 0 or -1 launches them one by one.  nrhs > 1: b and x hold nrhs fields solved
    together (FP64), and the stats are a list of per-column dicts.  TMQCD_ENOCONV and TMQCD_EBREAKDOWN
    raise unless raise_on_noconv / raise_on_breakdown is False.  Returns (x, stats, return code)."""
    subset = FULL if op == MDAGM else EVEN
    if x_is_zero is None:
        x_is_zero = x is None
    if x is None:
        x = _bytes(spinor_bytes(prob, F64, subset, nrhs))
    if ws is None:
        ws = _bytes(workspace_bytes(prob, op, 1 | (1 << inner_prec), nrhs))
    gp = (ctypes.c_void_p * 3)(*[_ptr(U_packed.get(p)) for p in (F64, F32, F16)])
    o = CCgOpts(tol=tol, max_iter=max_iter, op=op, inner_prec=inner_prec, recon=recon,
                reliable_delta=reliable_delta, check_every=check_every, x_is_zero=int(x_is_zero),
                use_graph=int(use_graph), nrhs=int(nrhs))
    st = (CCgStats * max(1, nrhs))()
    rc = lib().tmqcd_cg(ctypes.byref(prob.c()), ctypes.byref(gp), _ptr(b), _ptr(x), ctypes.byref(o),
                        st, _ptr(ws), ws.numel(), _stream(stream))
    tolerated = (OK,) + (() if raise_on_noconv else (ENOCONV,)) + (() if raise_on_breakdown else (EBREAKDOWN,))
    if rc not in tolerated:
        raise TmqcdError(rc, "tmqcd_cg")
    stats = [s.as_dict() for s in st]
    return x, (stats if nrhs > 1 else stats[0]), rc


def bicgstab_workspace_bytes(prob: Problem, op=MHAT) -> int:
    return lib().tmqcd_bicgstab_workspace_bytes(ctypes.byref(prob.c()), op)


def bicgstab(prob: Problem, U_packed, b, x=None, *, x_is_zero=None, tol=1e-10, max_iter=10000, op=MHAT,
             recon=RECON18, check_every=0, ws=None, stream=None, raise_on_noconv=True):
    """Solve op x = b with BiCGStab, op = M (full fields) or MHAT (even fields); U_packed: FP64 links.

    x, x_is_zero as for cg (use_graph does not apply).  Returns (x, stats dict, return code)."""
    subset = FULL if op == M else EVEN
    if x_is_zero is None:
        x_is_zero = x is None
    if x is None:
        x = _bytes(spinor_bytes(prob, F64, subset))
    if ws is None:
        ws = _bytes(bicgstab_workspace_bytes(prob, op))
    o = CCgOpts(tol=tol, max_iter=max_iter, op=op, inner_prec=F64, recon=recon, reliable_delta=0.0,
                check_every=check_every, x_is_zero=int(x_is_zero))
    st = CCgStats()
    rc = lib().tmqcd_bicgstab(ctypes.byref(prob.c()), _ptr(U_packed), _ptr(b), _ptr(x), ctypes.byref(o),
                              ctypes.byref(st), _ptr(ws), ws.numel(), _stream(stream))
    if rc not in (OK, ENOCONV) or (rc == ENOCONV and raise_on_noconv):
        raise TmqcdError(rc, "tmqcd_bicgstab")
    return x, st.as_dict(), rc


def cg_batch(probs, U_packed, bs, xs=None, *, tol=1e-10, max_iter=10000, recon=RECON18, use_graph=True,
             check_every=0, ws=None, stream=None, raise_on_noconv=True, raise_on_breakdown=True):
    """FP64 CG on Mhat^dag Mhat for several lattices in one solve (packed FP64 even fields).

    A lattice that breaks down (TMQCD_EBREAKDOWN) stops alone; the others are solved.
    Returns (xs, [stats dict per lattice], return code)."""
    n = len(probs)
    cp = (CProblem * n)(*[p.c() for p in probs])
    if xs is None:
        xs = [_bytes(spinor_bytes(p, F64, EVEN)) for p in probs]
    if ws is None:
        ws = _bytes(lib().tmqcd_cg_batch_workspace_bytes(n, cp))
    arr = lambda ts: (ctypes.c_void_p * n)(*[_ptr(t) for t in ts])
    o = CCgOpts(tol=tol, max_iter=max_iter, op=MHATDAGMHAT, inner_prec=F64, recon=recon, reliable_delta=0.0,
                check_every=check_every, x_is_zero=1)
    st = (CCgStats * n)()
    rc = lib().tmqcd_cg_batch(n, cp, arr(U_packed), arr(bs), arr(xs), ctypes.byref(o), st, int(use_graph),
                              _ptr(ws), ws.numel(), _stream(stream))
    tolerated = (OK,) + (() if raise_on_noconv else (ENOCONV,)) + (() if raise_on_breakdown else (EBREAKDOWN,))
    if rc not in tolerated:
        raise TmqcdError(rc, "tmqcd_cg_batch")
    return xs, [s.as_dict() for s in st], rc


def tune(prob: Problem, U_packed, prec=F64, recon=RECON18, stream=None):
    """Tune the hop launch shapes for this problem; returns one dict per kernel class."""
    ws = _bytes(lib().tmqcd_tune_workspace_bytes(ctypes.byref(prob.c()), prec))
    res = (CTuneResult * 3)()
    _check(lib().tmqcd_tune(ctypes.byref(prob.c()), _ptr(U_packed), prec, recon, _ptr(ws), ws.numel(), res,
                            _stream(stream)), "tmqcd_tune")
    return [r.as_dict() for r in res]


def tune_save(path: str):
    _check(lib().tmqcd_tune_save(str(path).encode()), "tmqcd_tune_save")


def tune_load(path: str):
    _check(lib().tmqcd_tune_load(str(path).encode()), "tmqcd_tune_load")


def hbm_probe(src, dst=None, xor_out=None, grid=2048, stream=None):
    """Copy src (uint8 device tensor, 16-byte multiple) to dst, or with dst None stream it with 16-byte reads,
    xoring its 32-bit words into xor_out (an int32 device tensor of one element)."""
    _check(lib().tmqcd_hbm_probe(_ptr(src), _ptr(dst), src.numel(), grid, _ptr(xor_out), _stream(stream)),
           "tmqcd_hbm_probe")


def tune_clear():
    lib().tmqcd_tune_clear()


def tune_set(prob: Problem, prec, recon, kernel_class, block, order, nrhs=1, group=0):
    """Pin the launch shape (block 128/256, order 0..5; class 3: multi-RHS with nrhs and group) for this problem."""
    _check(lib().tmqcd_tune_set(ctypes.byref(prob.c()), prec, recon, kernel_class, nrhs, block, order, group),
           "tmqcd_tune_set")


def tune_mrhs(prob: Problem, U_packed, nrhs, prec=F64, recon=RECON18, stream=None):
    """Tune the block order of the multi-RHS hop for nrhs right-hand sides; returns the result dict."""
    ws = _bytes(lib().tmqcd_tune_mrhs_workspace_bytes(ctypes.byref(prob.c()), prec, nrhs))
    res = CTuneResult()
    _check(lib().tmqcd_tune_mrhs(ctypes.byref(prob.c()), _ptr(U_packed), prec, recon, nrhs, _ptr(ws), ws.numel(),
                                 ctypes.byref(res), _stream(stream)), "tmqcd_tune_mrhs")
    return res.as_dict()


def _mom(prob: Problem, out, like):
    import torch
    if out is None:
        out = torch.empty((prob.volume, 4, 8), dtype=torch.float64, device=like.device)
    return out


def force_workspace_bytes(prob: Problem) -> int:
    return lib().tmqcd_force_workspace_bytes(ctypes.byref(prob.c()))


def force(prob: Problem, U_packed, X, Y=None, recon=RECON18, out=None, scale=1.0, accumulate=False, ws=None,
          stream=None):
    """scale * dS_f/dw^a (float64 device tensor (V, 4, 8)) from packed FP64 full fields X and Y = M X
    (Y None: computed by the library into ws, allocated when None); with accumulate the result is
    added to `out`."""
    out = _mom(prob, out, X)
    if Y is None and ws is None:
        ws = _bytes(force_workspace_bytes(prob), X.device)
    nbytes = 0 if ws is None else ws.numel() * ws.element_size()
    _check(lib().tmqcd_force(ctypes.byref(prob.c()), _ptr(U_packed), recon, _ptr(X), _ptr(Y), _ptr(out),
                             float(scale), int(accumulate), _ptr(ws), nbytes, _stream(stream)), "tmqcd_force")
    return out


def force_eo_workspace_bytes(prob: Problem) -> int:
    return lib().tmqcd_force_eo_workspace_bytes(ctypes.byref(prob.c()))


def force_eo(prob: Problem, U_packed, X_e, recon=RECON18, out=None, scale=1.0, accumulate=False, ws=None,
             stream=None):
    """scale * dS_f^eo/dw^a (float64 device tensor (V, 4, 8)) of phi_e^+ (Mhat^+ Mhat)^{-1} phi_e from the
    packed FP64 even field X_e = (Mhat^+ Mhat)^{-1} phi_e; with accumulate the result is added to `out`."""
    out = _mom(prob, out, X_e)
    if ws is None:
        ws = _bytes(force_eo_workspace_bytes(prob), X_e.device)
    _check(lib().tmqcd_force_eo(ctypes.byref(prob.c()), _ptr(U_packed), recon, _ptr(X_e), _ptr(out), float(scale),
                                int(accumulate), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "tmqcd_force_eo")
    return out


def gauge_force(prob: Problem, U_packed, beta, out=None, scale=1.0, accumulate=False, stream=None):
    """scale * dS_g/dw^a of the Wilson plaquette action (FP64 RECON18 links)."""
    out = _mom(prob, out, U_packed)
    _check(lib().tmqcd_gauge_force(ctypes.byref(prob.c()), _ptr(U_packed), float(beta), _ptr(out), float(scale),
                                   int(accumulate), _stream(stream)), "tmqcd_gauge_force")
    return out


def gauge_force_tlsym_workspace_bytes(prob: Problem) -> int:
    return lib().tmqcd_gauge_force_tlsym_workspace_bytes(ctypes.byref(prob.c()))


def gauge_force_tlsym(prob: Problem, U_packed, beta, c1, out=None, scale=1.0, accumulate=False, ws=None, stream=None):
    """scale * dS_g/dw^a of the tree-level Symanzik action with rectangle coefficient c1, c0 = 1 - 8 c1
    (FP64 RECON18 links); ws: the staple-field workspace (allocated when None and c1 != 0)."""
    out = _mom(prob, out, U_packed)
    if ws is None and c1 != 0:
        ws = _bytes(gauge_force_tlsym_workspace_bytes(prob), U_packed.device)
    nbytes = 0 if ws is None else ws.numel() * ws.element_size()
    _check(lib().tmqcd_gauge_force_tlsym(ctypes.byref(prob.c()), _ptr(U_packed), float(beta), float(c1), _ptr(out),
                                         float(scale), int(accumulate), _ptr(ws), nbytes, _stream(stream)),
           "tmqcd_gauge_force_tlsym")
    return out


def heatbath(prob: Problem, U_packed, beta, seed, sweep, prec=F64, stream=None):
    """One heatbath sweep of the Wilson action, in place on packed RECON18 links of precision prec (F64/F32)."""
    _check(lib().tmqcd_heatbath(ctypes.byref(prob.c()), _ptr(U_packed), prec, float(beta),
                                int(seed) & (2 ** 64 - 1), int(sweep) & 0xFFFFFFFF, _stream(stream)), "tmqcd_heatbath")


def overrelax(prob: Problem, U_packed, prec=F64, stream=None):
    """One overrelaxation sweep, in place on packed RECON18 links of precision prec (F64/F32)."""
    _check(lib().tmqcd_overrelax(ctypes.byref(prob.c()), _ptr(U_packed), prec, _stream(stream)), "tmqcd_overrelax")


def update_links(prob: Problem, U_packed, p, dt, stream=None):
    """U <- exp(i dt p^a T^a) U in place (FP64 RECON18 packed links)."""
    _check(lib().tmqcd_update_links(ctypes.byref(prob.c()), _ptr(U_packed), _ptr(p), float(dt), _stream(stream)),
           "tmqcd_update_links")
    return U_packed


def aux_workspace(prob: Problem):
    return _bytes(workspace_bytes(prob, -1, 1, 1))


def _result(n, like):
    import torch
    return torch.empty(n, dtype=torch.float64, device=like.device)


def plaquette(prob: Problem, U_packed, ws=None, out=None, stream=None):
    """Device tensor [sum_{x, mu<nu} Re Tr P_mu_nu(x)]."""
    ws = aux_workspace(prob) if ws is None else ws
    out = _result(1, U_packed) if out is None else out
    _check(lib().tmqcd_plaquette(ctypes.byref(prob.c()), _ptr(U_packed), _ptr(out), _ptr(ws), ws.numel(),
                                 _stream(stream)), "tmqcd_plaquette")
    return out


def rectangle(prob: Problem, U_packed, ws=None, out=None, stream=None):
    """Device tensor [sum_{x, mu != nu} Re Tr R_mu_nu(x)] over the 12 V rectangles."""
    ws = aux_workspace(prob) if ws is None else ws
    out = _result(1, U_packed) if out is None else out
    _check(lib().tmqcd_rectangle(ctypes.byref(prob.c()), _ptr(U_packed), _ptr(out), _ptr(ws), ws.numel(),
                                 _stream(stream)), "tmqcd_rectangle")
    return out


def momentum_norm2(prob: Problem, p, ws=None, out=None, stream=None):
    """Device tensor [sum p^2]."""
    ws = aux_workspace(prob) if ws is None else ws
    out = _result(1, p) if out is None else out
    _check(lib().tmqcd_momentum_norm2(ctypes.byref(prob.c()), _ptr(p), _ptr(out), _ptr(ws), ws.numel(),
                                      _stream(stream)), "tmqcd_momentum_norm2")
    return out


def dot(prob: Problem, x, y, subset=FULL, ws=None, out=None, stream=None):
    """Device tensor [Re, Im] of x^+ y for packed FP64 fields."""
    ws = aux_workspace(prob) if ws is None else ws
    out = _result(2, x) if out is None else out
    _check(lib().tmqcd_dot(ctypes.byref(prob.c()), _ptr(x), _ptr(y), subset, _ptr(out), _ptr(ws), ws.numel(),
                           _stream(stream)), "tmqcd_dot")
    return out


def delta_h(prob: Problem, U0, U1, p0, p1, phi, X0, X1, subset=FULL, beta=0.0, c1=0.0, ws=None, out=None,
            stream=None):
    """Device tensor [dH, kinetic, gauge, fermion] between (U0, p0, X0) and (U1, p1, X1), summed site by site
    in FP64 (packed FP64 RECON18 links, momenta (V, 4, 8), packed FP64 fields phi, X of `subset`)."""
    ws = aux_workspace(prob) if ws is None else ws
    out = _result(4, p0) if out is None else out
    _check(lib().tmqcd_delta_h(ctypes.byref(prob.c()), _ptr(U0), _ptr(U1), _ptr(p0), _ptr(p1), _ptr(phi), _ptr(X0),
                               _ptr(X1), subset, float(beta), float(c1), _ptr(out), _ptr(ws), ws.numel(),
                               _stream(stream)), "tmqcd_delta_h")
    return out
