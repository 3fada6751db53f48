"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and its host-only Clements helper agrees with the oracle's."""
import os
import re

import numpy as np
import pytest

from oracle import clements as oclem
from paper_2301_12814_amd import gbsmpo, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbs_mpo.h")

pytestmark = pytest.mark.skipif(not os.path.exists(gbsmpo.LIB_PATH),
                                reason="libgbsmpo.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:mpo|gbs)_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = gbsmpo.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("M,seed", [(2, 3), (5, 4), (8, 1), (32, 2), (64, 3)])
def test_clements_matches_oracle(M, seed):
    U = inputs.haar_unitary(M, seed)
    layers, phase = gbsmpo.clements(U)
    og, oph = oclem.decompose(U)
    ol = oclem.layers(M, og)
    assert len(layers) == len(ol)
    flat = [(int(s), t, p) for (S, T, P) in layers for s, t, p in zip(S, T, P)]
    oflat = [g for layer in ol for g in layer]
    assert [f[0] for f in flat] == [g[0] for g in oflat]
    assert np.allclose([f[1] for f in flat], [g[1] for g in oflat], atol=1e-12)
    dphi = np.angle(np.exp(1j * (np.array([f[2] for f in flat]) - np.array([g[2] for g in oflat]))))
    assert np.abs(dphi).max() < 1e-10
    # the library's own gates reconstruct U
    assert np.abs(oclem.reconstruct(M, flat, phase) - U).max() < 1e-11


def test_clements_rejects_non_unitary():
    U = np.eye(3, dtype=complex) * 1.1
    with pytest.raises(gbsmpo.GbsMpoError):
        gbsmpo.clements(U)
