"""The bandwidth probe: its copy reproduces the source bytes; its read xors every word (checked on the host)."""
import numpy as np
import pytest
import torch

from paper_1209_5942_amd import tmqcd as T

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes,grid", [(16, 1), (1 << 20, 64), ((1 << 24) + 48, 2048)])
def test_probe_copy_and_read(nbytes, grid):
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    a = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    keep = a.clone()
    c = torch.zeros_like(a)
    word = torch.zeros(1, dtype=torch.int32, device="cuda")
    T.hbm_probe(a, c, grid=grid)
    T.hbm_probe(a, xor_out=word, grid=grid)
    torch.cuda.synchronize()
    assert torch.equal(c, a) and torch.equal(a, keep)
    want = np.bitwise_xor.reduce(keep.cpu().numpy().view(np.uint32))
    assert int(word.cpu().numpy().view(np.uint32)[0]) == int(want)
