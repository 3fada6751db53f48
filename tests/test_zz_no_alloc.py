"""mpo_photon_marginals_noalloc (the entry point for callers that cannot
allocate device memory) against mpo_photon_marginals on the same state, two
calls in a row, the second on a smaller state: the static scratch array keeps
the last call's contents, so stale data from the first call must not leak
into the second.  Both run the same kernels in the same order, so the
results agree bit for bit."""
import numpy as np
import pytest

from paper_2301_12814_amd import gbsmpo, inputs

pytestmark = pytest.mark.gpu


def _evolved(M, d, chi, r, eta, seed, n_layers):
    g = gbsmpo.MPO(M, r, eta, d, chi)
    layers, _ = gbsmpo.clements(inputs.haar_unitary(M, seed))
    for L in layers[:n_layers]:
        g.apply_layer(*L)
    return g


def test_noalloc_marginals_match_allocating_entry_point():
    cases = [(16, 6, 64, 0.8, 0.5, 7, 6),     # larger state first
             (6, 4, 16, 0.6, 0.6, 8, 3)]      # then a smaller one
    for (M, d, chi, r, eta, seed, nl) in cases:
        print("noalloc case", M, d, chi, flush=True)
        with _evolved(M, d, chi, r, eta, seed, nl) as g:
            P0, t0 = g.marginals()
            P1, t1 = g.marginals_noalloc()
            assert P1.shape == (M, d)
            assert t1 == t0
            assert np.array_equal(P1, P0)

