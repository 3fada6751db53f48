"""GPU parity of the whole state: the library's Gamma and lambda (read back
through mpo_get_site / mpo_get_bond) contracted into the full density matrix
and compared entry by entry with the brute-force evolution rho -> U rho U^dag
(Sec. II, the vectorised unitary acting on ket and bra).  Full entries are
phase-sensitive, so these tests pin the output phase screen D and the
scatter's Gamma~ = V / lam (App. D), which the gauge-invariant readouts
(lambda, EE, marginals, trace) cannot see.
"""
import sys

import numpy as np
import pytest

from oracle import brute, clements as oclem, states
from paper_2301_12814_amd import gbsmpo, inputs
from tests.blocked import library_rho

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("M,d,r,eta,seed", [(3, 4, [0.7, 0.4, 0.9], 0.6, 11),
                                            (4, 3, [0.9, 0.0, 0.4, 0.7], 0.6, 12)])
def test_gpu_full_state_matches_brute_force(M, d, r, eta, seed):
    """chi above every rank (no truncation): after every layer and after the
    phase screen, the contracted library MPO equals the brute-force rho to
    1e-12 entrywise, and every Gamma entry outside the charge pattern is 0."""
    chi = 512
    U = inputs.haar_unitary(M, seed)
    layers, phase = gbsmpo.clements(U)
    og, oph = oclem.decompose(U)
    olayers = oclem.layers(M, og)
    rho = brute.product_rho([states.lossy_squeezed_rho(x, eta, d) for x in r])
    with gbsmpo.MPO(M, r, eta, d, chi) as g:
        got, outside = library_rho(g, M, d)
        assert outside == 0.0
        assert np.abs(got - rho).max() < 1e-12, "initial state"
        for li, (S, T, P) in enumerate(layers):
            g.apply_layer(S, T, P)
            for (k, th, ph) in olayers[li]:
                rho = brute.apply_gate(rho, k, th, ph)
            got, outside = library_rho(g, M, d)
            say("full state", M, d, "layer", li, "err", float(np.abs(got - rho).max()))
            assert outside == 0.0, li
            assert np.abs(got - rho).max() < 1e-12, li
        g.apply_phases(phase)
        rho = brute.apply_phases(rho, oph)
        got, _ = library_rho(g, M, d)
        err = float(np.abs(got - rho).max())
        # the screen with the opposite sign must be visibly different, so the
        # comparison above really sees the phases
        wrong = brute.apply_phases(brute.apply_phases(rho, -oph), -oph)
        say("after phase screen, err", err, "opposite-sign distance",
            float(np.abs(got - wrong).max()))
        assert err < 1e-12
        assert np.abs(got - wrong).max() > 1e-3


def test_gpu_phase_screen_on_product_state():
    """The phase screen alone on an input with coherences (squeezed modes):
    rho[m, m'] picks up e^{i phi (m - m')} per mode, entry by entry."""
    M, d = 3, 5
    r, eta = [0.8, 0.5, 1.0], 0.7
    ph = np.array([0.4, -1.3, 2.2])
    rho = brute.product_rho([states.lossy_squeezed_rho(x, eta, d) for x in r])
    with gbsmpo.MPO(M, r, eta, d, 256) as g:
        g.apply_phases(ph)
        got, _ = library_rho(g, M, d)
    n = np.arange(d)
    want = rho.copy()
    for j in range(M):
        f = np.exp(1j * ph[j] * (n[:, None] - n[None, :]))
        shape = [1] * (2 * M)
        shape[j], shape[M + j] = d, d
        want = want * f.reshape(shape)
    assert np.abs(got - want).max() < 1e-13


def test_gpu_identity_gates_keep_the_state():
    """Identity beam splitters (theta = phi = 0) on an exact Vidal state: the
    charges of every bond are bit-identical and the full rho is unchanged.
    The two-site update recomputes lambda by an SVD (App. D), which is
    backward stable: each value may move by a few units of rounding of the
    bond's largest value, so lambda is compared to 1e-13 of the bond maximum."""
    M, d = 4, 3
    r = [0.7, 0.3, 0.5, 0.9]
    with gbsmpo.MPO(M, r, 0.6, d, 512) as g:
        before = [g.bond(b) for b in range(M + 1)]
        rho0, _ = library_rho(g, M, d)
        g.apply_layer([0, 2], [0.0] * 2, [0.0] * 2)
        g.apply_layer([1], [0.0], [0.0])
        worst = 0.0
        for b in range(M + 1):
            lam, ch = g.bond(b)
            assert np.array_equal(ch, before[b][1]), b
            e = float(np.abs(lam - before[b][0]).max() / before[b][0].max())
            worst = max(worst, e)
        rho1, _ = library_rho(g, M, d)
        say("identity gates: worst lambda change / bond max", worst,
            "rho change", float(np.abs(rho1 - rho0).max()))
        assert worst < 1e-13
        assert np.abs(rho1 - rho0).max() < 1e-13
