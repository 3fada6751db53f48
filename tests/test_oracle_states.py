"""Pins of the oracle's per-mode input states (squeezed vacuum, App. C; pure
loss Kraus channel, App. B) against closed forms and an independent path."""
import math

import numpy as np
import pytest

from oracle import fock, states
from tests import closed_forms as cf

CASES = [(0.5, 0.5), (0.8, 0.398098197), (0.9, 0.3), (1.2, 0.8), (0.3, 1.0), (1.0, 0.25)]


@pytest.mark.parametrize("r,eta", CASES)
def test_diagonal_matches_generating_function(r, eta):
    d = 40
    rho = states.lossy_squeezed_rho(r, eta, d)
    P = cf.lossy_squeezed_distribution(r, eta, d)
    assert np.abs(np.diag(rho) - P).max() < 1e-13


@pytest.mark.parametrize("r,eta", CASES)
def test_trace_mean_variance_purity_uncropped(r, eta):
    n_int = states.internal_cutoff(r, 8)
    psi = states.squeezed_vacuum(r, n_int)
    rho = states.apply_loss(np.outer(psi, psi), eta)
    n = np.arange(n_int)
    p = np.diag(rho)
    s2, c2 = math.sinh(r) ** 2, math.cosh(r) ** 2
    assert abs(p.sum() - 1) < 1e-13
    mean = (n * p).sum()
    assert abs(mean - eta * s2) < 1e-12
    var = (n * n * p).sum() - mean ** 2
    # binomial thinning of the squeezed-vacuum variance 2 s^2 c^2
    assert abs(var - (2 * eta * eta * s2 * c2 + eta * (1 - eta) * s2)) < 1e-10
    N, A = cf.lossy_squeezed_moments(r, eta)
    assert abs(np.sum(rho * rho) - cf.gaussian_purity(N, A)) < 1e-12


@pytest.mark.parametrize("r,eta", CASES[:3])
def test_structure_parity_symmetry(r, eta):
    rho = states.lossy_squeezed_rho(r, eta, 12)
    assert np.abs(rho - rho.T).max() < 1e-16
    m, n = np.indices(rho.shape)
    assert np.all(rho[(m - n) % 2 == 1] == 0)       # App. B: odd entries vanish
    assert np.all(np.linalg.eigvalsh(rho) > -1e-15)


def test_pure_state_when_no_loss():
    r = 0.7
    rho = states.lossy_squeezed_rho(r, 1.0, 20)
    P = cf.lossy_squeezed_distribution(r, 1.0, 20)
    assert np.abs(np.diag(rho) - P).max() < 1e-14
    n_int = states.internal_cutoff(r, 20)
    psi = states.squeezed_vacuum(r, n_int)
    assert abs(np.sum(psi ** 2) - 1) < 1e-14
    assert psi[2] > 0            # + tanh(r) sign as printed in App. C


def test_vacuum():
    rho = states.lossy_squeezed_rho(0.0, 0.4, 5)
    ref = np.zeros((5, 5))
    ref[0, 0] = 1
    assert np.array_equal(rho, ref)


def test_loss_equals_beam_splitter_with_vacuum_environment():
    """Independent path: loss = mixing with a vacuum mode on a beam splitter of
    transmission eta, then tracing the environment out."""
    r, eta, n = 0.6, 0.55, 24
    psi = states.squeezed_vacuum(r, n)
    th = math.acos(math.sqrt(eta))
    T = fock.bs_matrix(th, 0.0)
    # two-mode input |psi> (x) |0>, restricted to total photons < n
    out = np.zeros((n, n), dtype=complex)        # amplitude [i1, i2]
    for j1 in range(n):
        if psi[j1] == 0:
            continue
        blk = fock.fock_block(T, j1)             # total photons = j1
        for i1 in range(j1 + 1):
            out[i1, j1 - i1] += blk[i1, j1] * psi[j1]
    rho_bs = out @ out.conj().T                  # trace over mode 2
    rho_k = states.apply_loss(np.outer(psi, psi), eta)
    assert np.abs(rho_bs - rho_k).max() < 1e-13
