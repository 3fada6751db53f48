"""Pins of the oracle's interferometer decomposition (App. A M-layer array)."""
import math

import numpy as np
import pytest

from oracle import clements
from paper_2301_12814_amd import inputs


@pytest.mark.parametrize("M,seed", [(2, 0), (3, 5), (8, 1), (13, 7), (32, 2)])
def test_reconstruct(M, seed):
    U = inputs.haar_unitary(M, seed)
    gates, phases = clements.decompose(U)
    assert len(gates) == M * (M - 1) // 2
    assert np.abs(clements.reconstruct(M, gates, phases) - U).max() < 1e-12
    L = clements.layers(M, gates)
    assert len(L) == (M if M > 2 else 1)
    for layer in L:
        sites = [g[0] for g in layer]
        assert len(set(sites) | {s + 1 for s in sites}) == 2 * len(sites)
    for (m, th, ph) in gates:
        assert 0 <= th <= math.pi / 2 + 1e-15
        assert -math.pi < ph <= math.pi


def test_haar_unitary_is_unitary_and_seeded():
    U = inputs.haar_unitary(16, 3)
    assert np.abs(U @ U.conj().T - np.eye(16)).max() < 1e-13
    assert np.array_equal(U, inputs.haar_unitary(16, 3))
