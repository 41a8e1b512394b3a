"""Pins for the oracle's compressed link formats (no GPU): exact round trips on SU(3), the byte counts of
the paper's Table 3, and the loss of accuracy near a first row (e^{i phi}, 0, 0) as 1/(|a2|^2 + |a3|^2)."""
import json
import os

import numpy as np
import pytest

from oracle import compress as C
from paper_1209_5942_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("eps", [0.1, 0.5, 2.0])
def test_round_trips_on_su3(eps):
    U = synth.random_links((4, 4, 2, 4), eps, 41).reshape(-1, 3, 3)
    assert np.abs(C.rec12_decode(U[:, :2, :]) - U).max() < 1e-14
    assert np.abs(C.rec10_decode(C.rec10_encode(U)) - U).max() < 1e-12
    assert np.abs(C.rec8_decode(C.rec8_encode(U)) - U).max() < 1e-12


def test_counts_match_table3():
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "memory_table.json")))
    U = synth.random_links((2, 2, 2, 2), 0.5, 42).reshape(-1, 3, 3)[:1]
    n10 = sum(2 * np.asarray(x).size if np.iscomplexobj(x) else np.asarray(x).size for x in C.rec10_encode(U))
    n8 = sum(2 * np.asarray(x).size if np.iscomplexobj(x) else np.asarray(x).size for x in C.rec8_encode(U))
    assert (n10, n8) == (10, 8)
    assert 4 * 8 * n10 == gold["U_REC10"] and 4 * 8 * n8 == gold["U_REC8"]


def test_accuracy_degrades_as_the_first_row_becomes_a_phase():
    rng = np.random.default_rng(43)
    errs = []
    for d in (1e-1, 1e-3, 1e-5):
        # a link whose first row is (e^{i phi} sqrt(1 - d^2), O(d), O(d)): rotate diag(phases) slightly
        base = np.diag(np.exp(1j * np.array([0.3, -1.1, 0.8])))
        h = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
        h = (h + h.conj().T) / 2
        w, v = np.linalg.eigh(h)
        U = (v @ np.diag(np.exp(1j * d * w)) @ v.conj().T) @ base
        U = U / np.linalg.det(U) ** (1 / 3)
        errs.append(np.abs(C.rec8_decode(C.rec8_encode(U[None]))[0] - U).max())
    assert errs[0] < 1e-13
    assert errs[2] > 1e3 * errs[0]       # at |a2|^2 + |a3|^2 ~ 1e-10 the rounding of a1 and c1 is magnified
