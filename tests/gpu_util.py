"""Shared helpers of the GPU parity tests: seeded inputs, device transfer, oracle mapping."""
import numpy as np

from oracle import dirac as D
from paper_1209_5942_amd import synth
from paper_1209_5942_amd import tmqcd as T

BC_AP = (1, 1, 1, -1)
BC_TWIST = (np.exp(0.3j), np.exp(0.7j), -1.0, np.exp(1.1j))

# allowed relative L2 error against the FP64 oracle, per storage precision
TOL = {T.F64: 1e-12, T.F32: 5e-6, T.F16: 5e-3}

SUBSET_SITES = {T.FULL: 1, T.EVEN: 2, T.ODD: 2}


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.cpu().numpy()


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_op(op, U, psi, dims, kappa, mu, bc):
    """Oracle counterpart of a tmqcd op on canonical inputs of the op's input subset."""
    name = {v: k for k, v in T.OPS.items()}[op]
    return D.apply_op(name, U, psi, dims, kappa, mu, bc)


def n_sites(prob, subset):
    return prob.volume // SUBSET_SITES[subset]


_CACHE = {}


def cached_fields(dims, eps, seed, kappa, mu, bc=BC_AP):
    """One Fields object per argument set for the whole session (large lattices are slow to draw)."""
    key = (tuple(dims), eps, seed, kappa, mu, tuple(complex(b) for b in bc))
    if key not in _CACHE:
        _CACHE[key] = Fields(dims, eps, seed, kappa, mu, bc)
    return _CACHE[key]


class Fields:
    """Seeded gauge field and a Gaussian spinor of each subset, on host and device."""

    def __init__(self, dims, eps, seed, kappa, mu, bc=BC_AP):
        self.prob = T.Problem(dims, kappa, mu, bc)
        self.dims, self.kappa, self.mu, self.bc = dims, kappa, mu, bc
        self.U = synth.random_links(dims, eps, seed)
        self.U_dev = dev(self.U.reshape(-1, 4, 3, 3))
        self._packed = {}

    def gauge(self, prec, recon):
        key = (prec, recon)
        if key not in self._packed:
            self._packed[key] = T.pack_gauge(self.prob, self.U_dev, prec, recon)
        return self._packed[key]

    def spinor(self, subset, seed, nrhs=None):
        return synth.gaussian_spinor(n_sites(self.prob, subset), seed, nrhs)
