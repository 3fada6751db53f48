"""Pins of the oracle's two-mode Fock beam splitter (App. B transform, Eq. kun)."""
import math

import numpy as np
import pytest

from oracle import fock

ANGLES = [(0.3, 0.0), (0.7, 1.1), (1.2, -2.5), (math.pi / 4, math.pi / 3)]


@pytest.mark.parametrize("theta,phi", ANGLES)
def test_single_photon_amplitudes_are_T(theta, phi):
    T = fock.bs_matrix(theta, phi)
    U = fock.fock_bs(T, 3)
    assert abs(U[1, 0, 1, 0] - T[0, 0]) < 1e-15
    assert abs(U[0, 1, 1, 0] - T[1, 0]) < 1e-15
    assert abs(U[1, 0, 0, 1] - T[0, 1]) < 1e-15
    assert abs(U[0, 1, 0, 1] - T[1, 1]) < 1e-15


@pytest.mark.parametrize("theta,phi", ANGLES)
def test_eq_kun_special_case(theta, phi):
    """Input (n, 0): amplitude sqrt(binom(n, k)) T11^k T21^(n-k) (App. B, Eq. kun
    with cos/sin replaced by the first column of T)."""
    T = fock.bs_matrix(theta, phi)
    n = 7
    U = fock.fock_bs(T, n + 1)
    for k in range(n + 1):
        ref = math.sqrt(math.comb(n, k)) * T[0, 0] ** k * T[1, 0] ** (n - k)
        assert abs(U[k, n - k, n, 0] - ref) < 1e-13


@pytest.mark.parametrize("theta,phi", ANGLES)
def test_total_number_blocks_unitary(theta, phi):
    T = fock.bs_matrix(theta, phi)
    for n in range(0, 23):
        B = fock.fock_block(T, n)
        assert np.abs(B @ B.conj().T - np.eye(n + 1)).max() < 2e-12


def test_group_homomorphism():
    """U(T1 T2) = U(T1) U(T2) on every photon-number block: catches transposed
    or conjugated index conventions."""
    T1 = fock.bs_matrix(0.4, 0.9)
    T2 = fock.bs_matrix(1.1, -0.3)
    for n in range(0, 12):
        lhs = fock.fock_block(T1 @ T2, n)
        rhs = fock.fock_block(T1, n) @ fock.fock_block(T2, n)
        assert np.abs(lhs - rhs).max() < 1e-12


def test_special_angles():
    d = 6
    # theta = 0: phases e^{i phi j1} only
    phi = 0.77
    U = fock.fock_bs(fock.bs_matrix(0.0, phi), d)
    for i1 in range(d):
        for i2 in range(d):
            assert abs(U[i1, i2, i1, i2] - np.exp(1j * phi * i1)) < 1e-14
    # theta = pi/2, phi = 0: a1^dag -> a2^dag, a2^dag -> -a1^dag
    U = fock.fock_bs(fock.bs_matrix(math.pi / 2, 0.0), d)
    for j1 in range(d):
        for j2 in range(d):
            assert abs(U[j2, j1, j1, j2] - (-1) ** j2) < 1e-13


def test_cutoff_restriction_is_subblock():
    d = 4
    T = fock.bs_matrix(0.5, 0.2)
    U = fock.fock_bs(T, d)
    n = 5                                        # > d-1: truncated block
    B = fock.fock_block(T, n)
    for i1 in range(d):
        for j1 in range(d):
            if 0 <= n - i1 < d and 0 <= n - j1 < d:
                assert abs(U[i1, n - i1, j1, n - j1] - B[i1, j1]) < 1e-14
