"""The C interface on the host (no GPU): the library loads, exports every entry
point the header declares, reports packed sizes that match the paper's memory
table, and rejects bad arguments before making any HIP call."""
import ctypes
import json
import os
import re

import pytest

from paper_1209_5942_amd import tmqcd as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L(built_lib):
    return T.lib()


def test_header_symbols_exported(L):
    header = open(os.path.join(ROOT, "include", "tmqcd.h")).read()
    declared = set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\**(tmqcd_[a-z_0-9]+)\(", header, re.M))
    assert declared == set(T.ENTRY_POINTS)
    for name in declared:
        assert hasattr(L, name), name


def test_sizes_match_paper_memory_table(L):
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "memory_table.json")))
    prob = T.Problem((8, 8, 8, 8), 0.15, 0.0)       # V/2 is a multiple of 64: no padding
    v = prob.volume
    assert T.spinor_bytes(prob, T.F64, T.FULL) == gold["phi"] * v
    assert T.spinor_bytes(prob, T.F64, T.EVEN) == gold["phi_eo"] * v
    assert T.gauge_bytes(prob, T.F64, T.RECON18) == gold["U"] * v
    assert T.gauge_bytes(prob, T.F64, T.RECON12) == gold["U_REC12"] * v
    assert T.gauge_bytes(prob, T.F64, T.RECON10) == gold["U_REC10"] * v
    assert T.gauge_bytes(prob, T.F64, T.RECON8) == gold["U_REC8"] * v
    for rec, key in ((T.RECON10, "U_REC10"), (T.RECON8, "U_REC8")):
        assert T.gauge_bytes(prob, T.F32, rec) == gold[key] * v // 2
        assert T.gauge_bytes(prob, T.F16, rec) == gold[key] * v // 4
    # lower precisions halve and quarter the storage (FP16 spinors carry one FP32 scale per site)
    assert T.spinor_bytes(prob, T.F32, T.FULL) == gold["phi"] * v // 2
    assert T.spinor_bytes(prob, T.F16, T.FULL) == gold["phi"] * v // 4 + 4 * v
    assert T.gauge_bytes(prob, T.F32, T.RECON12) == gold["U_REC12"] * v // 2
    assert T.spinor_bytes(prob, T.F64, T.FULL, nrhs=12) == 12 * gold["phi"] * v


def test_ragged_volume_is_padded_to_a_wavefront(L):
    prob = T.Problem((6, 2, 2, 2), 0.15, 0.0)       # V/2 = 24 -> padded to 64
    assert T.spinor_bytes(prob, T.F64, T.EVEN) == 12 * 16 * 64
    assert T.workspace_bytes(prob, T.MHATDAGMHAT, 1 | 2 | 4) > 0


@pytest.mark.parametrize("dims", [(3, 4, 4, 4), (4, 4, 4, 1), (0, 4, 4, 4), (4, 4, 6, 5)])
def test_bad_extents_rejected(L, dims):
    prob = T.Problem(dims, 0.15, 0.0)
    assert T.gauge_bytes(prob) == 0
    rc = L.tmqcd_dslash(ctypes.byref(prob.c()), 256, 512, 1 << 20, T.M, T.F64, T.RECON18, 1, None, 0, None)
    assert rc == T.EINVAL


def _dslash(L, prob, U, inp, out, op=T.M, prec=T.F64, recon=T.RECON18, nrhs=1, ws=None, wsb=0):
    return L.tmqcd_dslash(ctypes.byref(prob.c()), U, inp, out, op, prec, recon, nrhs, ws, wsb, None)


def test_dslash_argument_errors(L):
    prob = T.Problem((4, 4, 4, 4), 0.15, 0.01)
    fb = T.spinor_bytes(prob, T.F64, T.FULL)
    U, a, b = 1 << 30, 1 << 32, 1 << 34              # never dereferenced: every call fails validation
    assert _dslash(L, prob, None, a, b) == T.EINVAL
    assert _dslash(L, prob, U, a, b, op=99) == T.EINVAL
    assert _dslash(L, prob, U, a, b, prec=3) == T.EINVAL
    assert _dslash(L, prob, U, a, b, recon=4) == T.EINVAL
    assert _dslash(L, prob, U, a, b, recon=-1) == T.EINVAL
    assert _dslash(L, prob, U, a, b, nrhs=0) == T.EINVAL
    assert _dslash(L, prob, U, a, b, nrhs=17) == T.EINVAL
    assert _dslash(L, prob, U, a + 8, b) == T.EALIGN
    assert _dslash(L, prob, U, a, a + fb - 256) == T.EALIAS
    assert _dslash(L, prob, U, a, b, op=T.MHAT, ws=None) == T.EWORKSPACE
    need = T.workspace_bytes(prob, T.MHAT, 1)
    assert _dslash(L, prob, U, a, b, op=T.MHAT, ws=1 << 36, wsb=need - 1) == T.EWORKSPACE
    assert _dslash(L, prob, U, a, b, op=T.MHAT, ws=a, wsb=need) == T.EALIAS


def test_cg_argument_errors(L):
    prob = T.Problem((4, 4, 4, 4), 0.15, 0.01)
    gp = (ctypes.c_void_p * 3)(1 << 30, None, None)
    st = T.CCgStats()

    def call(**kw):
        o = dict(tol=1e-10, max_iter=100, op=T.MHATDAGMHAT, inner_prec=T.F64, recon=0, reliable_delta=0.0,
                 check_every=0, x_is_zero=1)
        ws = kw.pop("ws", 1 << 36)
        wsb = kw.pop("wsb", 1 << 30)
        b = kw.pop("b", 1 << 32)
        x = kw.pop("x", 1 << 34)
        o.update(kw)
        return L.tmqcd_cg(ctypes.byref(prob.c()), ctypes.byref(gp), b, x, ctypes.byref(T.CCgOpts(**o)),
                          ctypes.byref(st), ws, wsb, None)

    assert call(op=T.M) == T.EINVAL
    assert call(tol=0.0) == T.EINVAL
    assert call(max_iter=0) == T.EINVAL
    assert call(use_graph=2) == T.EINVAL
    assert call(use_graph=-2) == T.EINVAL
    assert call(inner_prec=T.F32) == T.EINVAL          # no FP32 gauge field given
    assert call(reliable_delta=1.5) == T.EINVAL
    assert call(x=(1 << 32) + 256) == T.EALIAS
    assert call(ws=None) == T.EWORKSPACE
    assert call(wsb=1024) == T.EWORKSPACE
    assert call(b=(1 << 32) + 4) == T.EALIGN
    # several right-hand sides: FP64 only, no graph, up to 16; b and x span nrhs fields each
    assert call(nrhs=17) == T.EINVAL
    assert call(nrhs=-1) == T.EINVAL
    gp2 = (ctypes.c_void_p * 3)(1 << 30, 1 << 31, None)
    o = dict(tol=1e-10, max_iter=100, op=T.MHATDAGMHAT, inner_prec=T.F32, recon=0, reliable_delta=0.0,
             check_every=0, x_is_zero=1, nrhs=2)
    assert L.tmqcd_cg(ctypes.byref(prob.c()), ctypes.byref(gp2), 1 << 32, 1 << 34, ctypes.byref(T.CCgOpts(**o)),
                      ctypes.byref(st), 1 << 36, 1 << 30, None) == T.EINVAL
    assert call(nrhs=2, use_graph=1) == T.EINVAL
    fe = T.spinor_bytes(prob, T.F64, T.EVEN)
    assert call(nrhs=2, x=(1 << 32) + fe) == T.EALIAS          # x overlaps the second column of b
    need1 = T.workspace_bytes(prob, T.MHATDAGMHAT, 1, 1)
    need2 = T.workspace_bytes(prob, T.MHATDAGMHAT, 1, 2)
    assert need2 > need1
    assert call(nrhs=2, wsb=need2 - 256) == T.EWORKSPACE


def test_pack_and_force_argument_errors(L):
    prob = T.Problem((4, 4, 4, 4), 0.15, 0.01)
    p = ctypes.byref(prob.c())
    assert L.tmqcd_pack_gauge(p, None, 1 << 30, 0, 0, None) == T.EINVAL
    assert L.tmqcd_pack_gauge(p, (1 << 30) + 8, 1 << 32, 0, 0, None) == T.EALIGN
    assert L.tmqcd_pack_spinor(p, 1 << 30, 1 << 30, 0, 0, 1, None) == T.EALIAS
    assert L.tmqcd_pack_spinor(p, 1 << 30, 1 << 32, 0, 5, 1, None) == T.EINVAL
    # X and dSdw are required; Y = NULL asks the call to form Y = M X in ws
    assert L.tmqcd_force(p, 1 << 30, 0, None, 1 << 33, 1 << 34, 1.0, 0, None, 0, None) == T.EINVAL
    assert L.tmqcd_force(p, 1 << 30, 0, 1 << 32, 1 << 33, None, 1.0, 0, None, 0, None) == T.EINVAL
    assert L.tmqcd_force(p, 1 << 30, 0, 1 << 32, 1 << 33, 1 << 34, 1.0, 2, None, 0, None) == T.EINVAL
    assert L.tmqcd_force(p, 1 << 30, 0, 1 << 32, 1 << 33, 1 << 32, 1.0, 0, None, 0, None) == T.EALIAS
    fb = T.spinor_bytes(prob, T.F64, T.FULL)
    assert L.tmqcd_force_workspace_bytes(p) == fb
    assert L.tmqcd_force(p, 1 << 30, 0, 1 << 32, None, 1 << 34, 1.0, 0, None, 0, None) == T.EWORKSPACE
    assert L.tmqcd_force(p, 1 << 30, 0, 1 << 32, None, 1 << 34, 1.0, 0, 1 << 36, fb - 1, None) == T.EWORKSPACE
    assert L.tmqcd_force(p, 1 << 30, 0, 1 << 32, None, 1 << 34, 1.0, 0, (1 << 36) + 16, fb, None) == T.EALIGN
    assert L.tmqcd_force(p, 1 << 30, 0, 1 << 32, None, 1 << 34, 1.0, 0, 1 << 32, fb, None) == T.EALIAS
    assert L.tmqcd_gauge_force(p, 1 << 30, float("nan"), 1 << 34, 1.0, 0, None) == T.EINVAL
    assert L.tmqcd_gauge_force(p, 1 << 30, 5.0, 1 << 30, 1.0, 0, None) == T.EALIAS
    assert L.tmqcd_update_links(p, 1 << 30, (1 << 34) + 4, 0.1, None) == T.EALIGN
    assert L.tmqcd_plaquette(p, 1 << 30, 1 << 34, None, 0, None) == T.EWORKSPACE
    ws = T.workspace_bytes(prob, -1, 1, 1)
    assert ws >= 8 * 2 * (prob.volume * 4 // 256)
    assert L.tmqcd_momentum_norm2(p, 1 << 30, 1 << 34, 1 << 36, 8, None) == T.EWORKSPACE
    assert L.tmqcd_dot(p, 1 << 30, 1 << 32, 7, 1 << 34, 1 << 36, ws, None) == T.EINVAL
    assert L.tmqcd_dot(p, 1 << 30, 1 << 32, T.FULL, 1 << 36, 1 << 36, ws, None) == T.EALIAS


def test_force_eo_argument_errors(L):
    prob = T.Problem((4, 4, 4, 4), 0.15, 0.01)
    p = ctypes.byref(prob.c())
    hb = T.spinor_bytes(prob, T.F64, T.EVEN)
    need = L.tmqcd_force_eo_workspace_bytes(p)
    assert need == 3 * hb
    bad = T.Problem((3, 4, 4, 4), 0.15, 0.01)
    assert L.tmqcd_force_eo_workspace_bytes(ctypes.byref(bad.c())) == 0
    U, X, out, ws = 1 << 30, 1 << 32, 1 << 34, 1 << 36

    def call(U=U, recon=T.RECON18, X=X, out=out, scale=1.0, acc=0, ws=ws, wsb=need):
        return L.tmqcd_force_eo(p, U, recon, X, out, scale, acc, ws, wsb, None)
    assert call(U=None) == T.EINVAL
    assert call(recon=5) == T.EINVAL
    assert call(X=None) == T.EINVAL
    assert call(out=None) == T.EINVAL
    assert call(scale=float("inf")) == T.EINVAL
    assert call(acc=2) == T.EINVAL
    assert call(X=X + 8) == T.EALIGN
    assert call(out=out + 8) == T.EALIGN
    assert call(ws=None) == T.EWORKSPACE
    assert call(wsb=need - 1) == T.EWORKSPACE
    assert call(ws=ws + 16) == T.EALIGN
    assert call(out=X) == T.EALIAS
    assert call(out=U) == T.EALIAS
    assert call(ws=X) == T.EALIAS
    assert call(ws=out) == T.EALIAS
    assert call(ws=U) == T.EALIAS
    assert L.tmqcd_force_eo(ctypes.byref(bad.c()), U, 0, X, out, 1.0, 0, ws, need, None) == T.EINVAL


def test_tlsym_and_rectangle_argument_errors(L):
    prob = T.Problem((4, 4, 4, 4), 0.15, 0.01)
    p = ctypes.byref(prob.c())
    U, out, w = 1 << 30, 1 << 34, 1 << 36
    need = L.tmqcd_gauge_force_tlsym_workspace_bytes(p)
    assert need == 3456 * prob.volume

    def call(U=U, beta=5.0, c1=-1 / 12, out=out, acc=0, ws=w, wsb=need):
        return L.tmqcd_gauge_force_tlsym(p, U, beta, c1, out, 1.0, acc, ws, wsb, None)
    assert call(U=None) == T.EINVAL
    assert call(c1=float("nan")) == T.EINVAL
    assert call(beta=float("inf")) == T.EINVAL
    assert call(acc=3) == T.EINVAL
    assert call(U=U + 16) == T.EALIGN
    assert call(out=U) == T.EALIAS
    assert call(ws=None) == T.EWORKSPACE
    assert call(wsb=need - 1) == T.EWORKSPACE
    assert call(ws=w + 16) == T.EALIGN
    assert call(ws=U) == T.EALIAS
    assert call(ws=out) == T.EALIAS
    ws = T.workspace_bytes(prob, -1, 1, 1)
    assert L.tmqcd_rectangle(p, None, out, 1 << 36, ws, None) == T.EINVAL
    assert L.tmqcd_rectangle(p, U, out, 1 << 36, 8, None) == T.EWORKSPACE
    assert L.tmqcd_rectangle(p, U, out + 4, 1 << 36, ws, None) == T.EALIGN
    assert L.tmqcd_rectangle(p, U, 1 << 36, 1 << 36, ws, None) == T.EALIAS


def test_bicgstab_argument_errors(L):
    prob = T.Problem((4, 4, 4, 4), 0.15, 0.01)
    p = ctypes.byref(prob.c())
    need = L.tmqcd_bicgstab_workspace_bytes(p, T.MHAT)
    assert need > 7 * T.spinor_bytes(prob, T.F64, T.EVEN)
    assert L.tmqcd_bicgstab_workspace_bytes(p, T.MDAGM) == 0
    assert L.tmqcd_bicgstab_workspace_bytes(p, T.M) > need
    st = T.CCgStats()

    def call(U=1 << 30, b=1 << 32, x=1 << 33, ws=1 << 36, wsb=need, **kw):
        o = dict(tol=1e-10, max_iter=100, op=T.MHAT, inner_prec=T.F64, recon=0, reliable_delta=0.0, check_every=0,
                 x_is_zero=1)
        o.update(kw)
        return L.tmqcd_bicgstab(p, U, b, x, ctypes.byref(T.CCgOpts(**o)), ctypes.byref(st), ws, wsb, None)
    assert call(op=T.MHATDAGMHAT) == T.EINVAL
    assert call(inner_prec=T.F32) == T.EINVAL
    assert call(tol=0.0) == T.EINVAL
    assert call(max_iter=0) == T.EINVAL
    assert call(recon=7) == T.EINVAL
    assert call(U=None) == T.EINVAL
    assert call(b=(1 << 32) + 8) == T.EALIGN
    assert call(x=1 << 32) == T.EALIAS
    assert call(ws=None) == T.EWORKSPACE
    assert call(wsb=need - 1) == T.EWORKSPACE
    assert call(ws=1 << 32) == T.EALIAS
    assert call(ws=1 << 30) == T.EALIAS


def test_heatbath_argument_errors(L):
    prob = T.Problem((4, 4, 4, 4), 0.15, 0.01)
    p = ctypes.byref(prob.c())
    assert L.tmqcd_heatbath(p, None, T.F64, 5.7, 1, 0, None) == T.EINVAL
    assert L.tmqcd_heatbath(p, 1 << 30, T.F16, 5.7, 1, 0, None) == T.EINVAL
    assert L.tmqcd_heatbath(p, 1 << 30, T.F64, -1.0, 1, 0, None) == T.EINVAL
    assert L.tmqcd_heatbath(p, 1 << 30, T.F32, float("nan"), 1, 0, None) == T.EINVAL
    assert L.tmqcd_heatbath(p, (1 << 30) + 8, T.F64, 5.7, 1, 0, None) == T.EALIGN
    assert L.tmqcd_overrelax(p, None, T.F64, None) == T.EINVAL
    assert L.tmqcd_overrelax(p, 1 << 30, 7, None) == T.EINVAL
    assert L.tmqcd_overrelax(p, (1 << 30) + 8, T.F32, None) == T.EALIGN
    bad = T.Problem((3, 4, 4, 4), 0.15, 0.01)
    assert L.tmqcd_heatbath(ctypes.byref(bad.c()), 1 << 30, T.F64, 5.7, 1, 0, None) == T.EINVAL


def test_error_strings(L):
    for code in (T.OK, T.EINVAL, T.EALIAS, T.EALIGN, T.ENOCONV, T.EBREAKDOWN, T.EHIP, T.EWORKSPACE):
        assert T.error_string(code) and "unknown" not in T.error_string(code)
    assert "unknown" in T.error_string(-99)


def test_tune_table_file_validation(L, tmp_path):
    bad = tmp_path / "bad.jsonl"
    bad.write_text("not json\n")
    assert L.tmqcd_tune_load(str(bad).encode()) == T.EINVAL
    other = tmp_path / "other.jsonl"
    other.write_text('{"arch": "gfx000", "class": 0, "prec": 0, "recon": 0, "dims": [4, 4, 4, 4], '
                     '"nrhs": 1, "block": 128, "order": 1, "group": 0, "us": 1.000}\n')
    assert L.tmqcd_tune_load(str(other).encode()) == T.EINVAL      # another architecture
    assert L.tmqcd_tune_load(str(tmp_path / "missing").encode()) == T.EINVAL
    prob = T.Problem((4, 4, 4, 4), 0.15, 0.0)
    assert T.lib().tmqcd_tune_workspace_bytes(ctypes.byref(prob.c()), 0) > 0
    res = (T.CTuneResult * 3)()
    assert L.tmqcd_tune(ctypes.byref(prob.c()), 1 << 30, 0, 0, None, 0, res, None) == T.EWORKSPACE
    assert L.tmqcd_tune(ctypes.byref(prob.c()), 1 << 30, 5, 0, 1 << 32, 1 << 30, res, None) == T.EINVAL


def test_tune_set_validation_and_roundtrip(L, tmp_path):
    prob = T.Problem((4, 4, 4, 6), 0.15, 0.0)
    p = ctypes.byref(prob.c())
    assert L.tmqcd_tune_set(p, 0, 0, 4, 1, 128, 1, 0) == T.EINVAL      # no class 4
    assert L.tmqcd_tune_set(p, 0, 0, 0, 1, 192, 1, 0) == T.EINVAL      # block size
    assert L.tmqcd_tune_set(p, 0, 0, 0, 1, 128, 6, 0) == T.EINVAL      # order
    assert L.tmqcd_tune_set(p, 5, 0, 0, 1, 128, 1, 0) == T.EINVAL      # precision
    assert L.tmqcd_tune_set(p, 0, 0, 0, 2, 128, 1, 0) == T.EINVAL      # single-RHS class with nrhs 2
    assert L.tmqcd_tune_set(p, 0, 0, 3, 1, 256, 1, 0) == T.EINVAL      # multi-RHS class with nrhs 1
    assert L.tmqcd_tune_set(p, 0, 0, 3, 17, 256, 1, 0) == T.EINVAL     # nrhs above 16
    assert L.tmqcd_tune_set(p, 0, 0, 3, 12, 128, 1, 0) == T.EINVAL     # multi-RHS kernel has 256 threads
    assert L.tmqcd_tune_set(p, 0, 0, 3, 12, 256, 1, 13) == T.EINVAL    # group above nrhs
    assert L.tmqcd_tune_set(p, 0, 0, 1, 1, 256, 1, 2) == T.EINVAL      # group on a single-RHS class
    try:
        assert L.tmqcd_tune_set(p, 0, 1, 2, 1, 128, 3, 0) == T.OK
        assert L.tmqcd_tune_set(p, 1, 0, 3, 12, 256, 2, 6) == T.OK
        path = tmp_path / "t.jsonl"
        assert L.tmqcd_tune_save(str(path).encode()) == T.OK
        lines = path.read_text().strip().splitlines()
        assert len(lines) == 2
        assert any('"class": 2' in l and '"nrhs": 1' in l and '"order": 3' in l for l in lines)
        assert any('"class": 3' in l and '"nrhs": 12' in l and '"order": 2' in l and '"group": 6' in l for l in lines)
        assert all('"dims": [4, 4, 4, 6]' in l for l in lines)
        assert L.tmqcd_tune_load(str(path).encode()) == T.OK
    finally:
        T.tune_clear()


def test_tune_mrhs_validation(L):
    prob = T.Problem((4, 4, 4, 4), 0.15, 0.0)
    p = ctypes.byref(prob.c())
    assert L.tmqcd_tune_mrhs_workspace_bytes(p, 0, 1) == 0
    assert L.tmqcd_tune_mrhs_workspace_bytes(p, 0, 12) > 12 * 2 * T.spinor_bytes(prob, 0, T.EVEN)
    res = T.CTuneResult()
    assert L.tmqcd_tune_mrhs(p, 1 << 30, 0, 0, 1, 1 << 32, 1 << 30, ctypes.byref(res), None) == T.EINVAL
    assert L.tmqcd_tune_mrhs(p, 1 << 30, 0, 0, 12, None, 0, ctypes.byref(res), None) == T.EWORKSPACE
    assert L.tmqcd_tune_mrhs(p, 1 << 30, 0, 0, 12, 8, 1 << 30, ctypes.byref(res), None) == T.EALIGN


def test_hbm_probe_validation(L):
    w = 1 << 34
    assert L.tmqcd_hbm_probe(None, None, 1 << 20, 64, w, None) == T.EINVAL
    assert L.tmqcd_hbm_probe(1 << 30, None, 0, 64, w, None) == T.EINVAL
    assert L.tmqcd_hbm_probe(1 << 30, None, 100, 64, w, None) == T.EINVAL        # not a multiple of 16
    assert L.tmqcd_hbm_probe(1 << 30, None, 1 << 20, 0, w, None) == T.EINVAL
    assert L.tmqcd_hbm_probe(1 << 30, None, 1 << 20, 64, None, None) == T.EINVAL   # read needs the xor word
    assert L.tmqcd_hbm_probe((1 << 30) + 8, None, 1 << 20, 64, w, None) == T.EALIGN
    assert L.tmqcd_hbm_probe(1 << 30, None, 1 << 20, 64, w + 2, None) == T.EALIGN
    assert L.tmqcd_hbm_probe(1 << 30, (1 << 30) + 4096, 1 << 20, 64, None, None) == T.EALIAS
    assert L.tmqcd_hbm_probe(1 << 30, None, 1 << 20, 64, (1 << 30) + 64, None) == T.EALIAS
