"""tmqcd_dslash_noalloc (temporaries in the library's static device scratch) against tmqcd_dslash
(a caller workspace): the same kernels, so bitwise the same output, on two calls in a row, the
second with a smaller lattice; every operator; and the host-side rejection of temporaries larger
than the scratch."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import BC_AP, BC_TWIST, Fields, dev
from paper_1209_5942_amd import synth
from paper_1209_5942_amd import tmqcd as T

ALL_OPS = [T.DSLASH_EO, T.DSLASH_OE, T.M, T.MDAG, T.MDAGM, T.MHAT, T.MHATDAG, T.MHATDAGMHAT]


def _pair(f, op, prec, recon, nrhs, seed):
    sub_in, sub_out = T.OP_SUBSETS[op]
    n = f.prob.volume // (1 if sub_in == T.FULL else 2)
    psi = np.stack([synth.gaussian_spinor(n, seed + k) for k in range(nrhs)]) if nrhs > 1 else \
        synth.gaussian_spinor(n, seed)
    inp = T.pack_spinor(f.prob, dev(psi), prec, sub_in, nrhs=nrhs)
    g = f.gauge(prec, recon)
    want = T.dslash(f.prob, g, inp, op, prec, recon, nrhs=nrhs)
    out = torch.full_like(want, 0x5A)
    T.dslash_noalloc(f.prob, g, inp, out, op, prec, recon, nrhs=nrhs)
    # the sites' values (the packed buffers' alignment padding is never written)
    return (T.unpack_spinor(f.prob, out, prec, sub_out, nrhs), T.unpack_spinor(f.prob, want, prec, sub_out, nrhs))


@pytest.mark.gpu
def test_noalloc_equals_workspace_call_twice_second_smaller():
    big = Fields((16, 16, 16, 32), 0.4, 3001, 0.155, 0.01, BC_AP)
    small = Fields((4, 4, 2, 6), 0.5, 3002, 0.16, 0.005, BC_TWIST)
    for f, seed in ((big, 3011), (small, 3012)):
        out, want = _pair(f, T.MHATDAGMHAT, T.F64, T.RECON18, 1, seed)
        assert torch.equal(out, want)


@pytest.mark.gpu
@pytest.mark.parametrize("op", ALL_OPS)
def test_noalloc_every_operator(op):
    f = Fields((8, 4, 4, 6), 0.5, 3003, 0.16, 0.005, BC_TWIST)
    for prec, recon, nrhs in ((T.F64, T.RECON18, 1), (T.F32, T.RECON12, 3), (T.F16, T.RECON8, 1)):
        out, want = _pair(f, op, prec, recon, nrhs, 3020 + op)
        assert torch.equal(out, want), (op, prec, recon, nrhs)


@pytest.mark.gpu
def test_noalloc_at_the_largest_fp64_mhatdagmhat_that_fits():
    """24^3 x 48 in FP64: the two odd temporaries (127 MB) fit the 128 MiB scratch."""
    prob = T.Problem((24, 24, 24, 48), 0.16, 0.005, BC_AP)
    assert 2 * T.spinor_bytes(prob, T.F64, T.ODD) <= T.lib().tmqcd_noalloc_scratch_bytes()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    g = T.pack_gauge(prob, torch.randn((prob.volume, 4, 3, 3), dtype=torch.complex128, device="cuda", generator=gen))
    inp = T.pack_spinor(prob, torch.randn((prob.volume // 2, 4, 3), dtype=torch.complex128, device="cuda",
                                          generator=gen), T.F64, T.EVEN)
    want = T.dslash(prob, g, inp, T.MHATDAGMHAT)
    out = torch.empty_like(want)
    T.dslash_noalloc(prob, g, inp, out, T.MHATDAGMHAT)
    assert torch.equal(T.unpack_spinor(prob, out, T.F64, T.EVEN), T.unpack_spinor(prob, want, T.F64, T.EVEN))


def test_noalloc_rejects_temporaries_beyond_the_scratch(built_lib):
    """Checked on the host before any device call (no GPU needed): 32^3 x 64 FP64 Mhat^+Mhat
    needs two 201 MB odd fields."""
    L = T.lib()
    prob = T.Problem((32, 32, 32, 64), 0.162, 0.003, BC_AP)
    cap = L.tmqcd_noalloc_scratch_bytes()
    assert cap == 128 << 20
    assert 2 * T.spinor_bytes(prob, T.F64, T.ODD) > cap
    rc = L.tmqcd_dslash_noalloc(ctypes.byref(prob.c()), 1 << 30, 1 << 34, 1 << 36, T.MHATDAGMHAT, T.F64, T.RECON18,
                                1, None)
    assert rc == T.ESCRATCH
    assert "scratch" in T.error_string(rc)
    rc = L.tmqcd_dslash_noalloc(ctypes.byref(prob.c()), 1 << 30, 1 << 34, 1 << 34, T.MHAT, T.F64, T.RECON18, 1, None)
    assert rc == T.EALIAS
    rc = L.tmqcd_dslash_noalloc(ctypes.byref(prob.c()), 1 << 30, 1 << 34, 1 << 36, 9, T.F64, T.RECON18, 1, None)
    assert rc == T.EINVAL
