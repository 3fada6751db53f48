"""Phase-sensitive pins of the oracle: the complex coherences of every output
mode against the Gaussian closed form (Sec. II: a linear-optics unitary maps
the input modes linearly; App. A: Haar interferometer as a beam-splitter mesh
plus an output phase screen), and the initial-state constants of the four
workloads against closed forms that share nothing with the oracle."""
import math

import numpy as np
import pytest

from oracle import brute, clements, mpo, states
from paper_2301_12814_amd import inputs
from tests import closed_forms as cf


def _reduced(rho_full, i):
    """Single-mode reduced density matrix of mode i of a tensor
    [m_1..m_M, m'_1..m'_M]."""
    M = rho_full.ndim // 2
    letters = "abcdefghijklmnop"
    ket = list(letters[:M])
    bra = list(letters[:M])
    ket[i], bra[i] = "x", "y"
    return np.einsum("".join(ket) + "".join(bra) + "->xy", rho_full)


def _run(kind, M, d, r, eta, seed, phase_sign=1.0):
    """Reduced states of every output mode after the whole Clements mesh and
    the output phase screen D (times phase_sign), from the brute-force
    density matrix or the oracle's dense Vidal MPO; returns (U, modes, trace,
    number of beam splitters)."""
    rhos = [states.lossy_squeezed_rho(x, eta, d) for x in r]
    U = inputs.haar_unitary(M, seed)
    gates, phases = clements.decompose(U)
    ph = phase_sign * np.asarray(phases)
    if kind == "brute":
        rho = brute.product_rho(rhos)
        for (k, th, p) in gates:
            rho = brute.apply_gate(rho, k, th, p)
        rho = brute.apply_phases(rho, ph)
        tr = brute.marginals(rho)[1]
    else:
        m = mpo.DenseMPO.product(rhos, 10 ** 6)
        for (k, th, p) in gates:
            m.apply_gate(k, th, p, 10 ** 6)
        m.apply_phases(ph)
        rho = m.to_dense()
        tr = m.marginals()[1]
    return U, [_reduced(rho, i) for i in range(M)], tr, len(gates)


# (kind, M, d, r, eta, Haar seed)
CASES = [("brute", 3, 12, [0.35, 0.2, 0.3], 0.5, 31),
         ("oracle", 2, 12, [0.45, 0.3], 0.5, 32)]


@pytest.mark.parametrize("kind,M,d,r,eta,seed", CASES)
def test_output_coherences_match_gaussian_closed_form(kind, M, d, r, eta, seed):
    """rho_i[n, n'] of every output mode, including the complex coherences
    (n - n' = 2, 4, ...) that only the beam-splitter phases and the output
    phase screen D fix, equals the Gaussian state with <b_i^dag b_i> and the
    complex <b_i b_i> computed from the Haar U itself (not from its
    decomposition).  Exact as d -> infinity.  At finite d each of the G gates
    drops the amplitude outside the cutoff, so the state differs from the
    untruncated one by at most the dropped amplitudes: 2 G sqrt(1 - Tr rho)
    bounds the gap.  The brute-force evolution pins brute.apply_phases; the
    oracle's dense MPO is pinned directly here and equals brute force to
    1e-13 in test_oracle_mpo."""
    U, red, tr, G = _run(kind, M, d, r, eta, seed)
    N, A = cf.output_mode_coherences(U, r, eta)
    bound = 2 * G * math.sqrt(max(1.0 - tr, 0.0)) + 1e-12
    assert bound < 1e-3
    for i in range(M):
        ref = cf.gaussian_rho(N[i], A[i], d)
        assert abs(ref[0, 2]) > 0.02                  # a coherence the phases decide
        assert np.abs(red[i] - ref).max() <= bound, i


@pytest.mark.parametrize("kind,M,d,r,eta,seed", CASES)
def test_wrong_phase_sign_is_detected(kind, M, d, r, eta, seed):
    """The pin above is sensitive to the sign of the output phase screen:
    the run with D replaced by conj(D) misses the closed form by far more
    than the truncation bound."""
    U, red, tr, G = _run(kind, M, d, r, eta, seed, phase_sign=-1.0)
    N, A = cf.output_mode_coherences(U, r, eta)
    worst = max(np.abs(red[i] - cf.gaussian_rho(N[i], A[i], d)).max() for i in range(M))
    assert worst > 1e-2


def test_per_mode_state_matches_squeezed_thermal_closed_form():
    """Every entry (not only the diagonal) of the per-mode input state after
    loss equals the squeezed thermal state with the same moments."""
    for r, eta, d in [(0.5, 0.5, 6), (0.9, 0.3, 8), (1.2, 0.8, 10), (1.0, 0.25, 10)]:
        N, A = cf.lossy_squeezed_moments(r, eta)
        assert np.abs(states.lossy_squeezed_rho(r, eta, d) - cf.gaussian_rho(N, A, d)).max() < 1e-13


# Initial-state constants of the four workloads, derived from the closed-form
# charge convolution before any code of this repository existed: trace of the
# cropped product state, and operator EE (bits) of the untruncated middle bond.
INITIAL_CONSTANTS = {
    # name: (M, r, eta, d, trace, mid-bond EE)
    "small": (8, 0.5, 0.5, 4, 0.981753625, 1.17925),
    "medium": (32, 0.8, inputs.eta_sqrt_scaling(32, 0.8), 8, 0.989731842, 4.59834),
    "large": (64, 0.9, 0.3, 8, 0.982602712, 5.77630),
    "serving-large": (96, 1.0, 0.25, 10, 0.993918220, 6.5559),
}


def _closed_form_mid_entropy(M, r, eta, d):
    """EE of the middle bond of the untruncated product state: the bond's
    Schmidt values squared are proportional to the 2-D convolution of
    |rho_j|^2 over the modes right of the bond (one Schmidt vector per
    charge), with rho_j the squeezed thermal closed form."""
    N, A = cf.lossy_squeezed_moments(r, eta)
    a2 = np.abs(cf.gaussian_rho(N, A, d)) ** 2
    w = np.ones((1, 1))
    for _ in range(M - M // 2):
        W = w.shape[0] + d - 1
        acc = np.zeros((W, W))
        for m_ in range(d):
            for mp in range(d):
                if a2[m_, mp] > 0:
                    acc[m_:m_ + w.shape[0], mp:mp + w.shape[1]] += a2[m_, mp] * w
        w = acc
    p = w[w > 0] / w.sum()
    return float(-(p * np.log2(p)).sum())


@pytest.mark.parametrize("name", list(INITIAL_CONSTANTS))
def test_initial_constants(name):
    M, r, eta, d, tr_ref, ee_ref = INITIAL_CONSTANTS[name]
    # trace: product of cropped per-mode traces from the photon generating function
    Pn = cf.lossy_squeezed_distribution(r, eta, d)
    tr_cf = float(Pn.sum()) ** M
    assert abs(tr_cf - tr_ref) < 1e-9
    rho1 = states.lossy_squeezed_rho(r, eta, d)
    assert abs(np.trace(rho1) ** M - tr_cf) < 1e-12
    ee_cf = _closed_form_mid_entropy(M, r, eta, d)
    assert abs(ee_cf - ee_ref) < 10 ** -(len(str(ee_ref).split(".")[1])) * 0.6
    if M <= 64:
        lam = np.array(list(mpo.product_lambdas([rho1] * M)[M // 2].values()))
        p = lam ** 2 / (lam ** 2).sum()
        p = p[p > 0]
        assert abs(float(-(p * np.log2(p)).sum()) - ee_cf) < 1e-12
