"""Two-mode Fock-space beam splitter (oracle, FP64).

Test infrastructure only (see ``oracle/__init__``).

A linear-optical element T (2x2 unitary) acts on creation operators as
a_j^dag -> sum_i T[i, j] a_i^dag (App. B, creation-operator transform).  The
Fock amplitude <i1, i2 | U | j1, j2> is the coefficient of
a1^dag^{i1} a2^dag^{i2} |0> / sqrt(i1! i2!) in
(T11 a1^dag + T21 a2^dag)^{j1} (T12 a1^dag + T22 a2^dag)^{j2} |0> / sqrt(j1! j2!),
expanded here term by term with the binomial theorem.  For an input (n, 0)
it reduces to the single-mode split of App. B, Eq. kun.

The matrix is built for photon numbers up to ``nmax`` per mode and then
restricted to the per-mode cutoff [0, d)^2; the restriction of a total-n
block with n > d-1 is a sub-block of a unitary and therefore not unitary.
"""
from __future__ import annotations

import math

import numpy as np


def bs_matrix(theta: float, phi: float) -> np.ndarray:
    """T(theta, phi) = [[e^{i phi} cos t, -sin t], [e^{i phi} sin t, cos t]]."""
    e = np.exp(1j * phi)
    return np.array([[e * math.cos(theta), -math.sin(theta)],
                     [e * math.sin(theta), math.cos(theta)]], dtype=complex)


def fock_amplitude(T: np.ndarray, i1: int, i2: int, j1: int, j2: int) -> complex:
    """<i1, i2 | U(T) | j1, j2> by the binomial expansion."""
    if i1 + i2 != j1 + j2:
        return 0.0j
    acc = 0.0j
    # k photons of input mode 1 go to output mode 1, i1 - k photons of input
    # mode 2 go to output mode 1.
    for k in range(0, j1 + 1):
        l = i1 - k
        if l < 0 or l > j2:
            continue
        acc += (math.comb(j1, k) * math.comb(j2, l)
                * T[0, 0] ** k * T[1, 0] ** (j1 - k)
                * T[0, 1] ** l * T[1, 1] ** (j2 - l))
    norm = math.sqrt(math.factorial(i1) * math.factorial(i2)
                     / (math.factorial(j1) * math.factorial(j2)))
    return acc * norm


def fock_bs(T: np.ndarray, d: int) -> np.ndarray:
    """U[i1, i2, j1, j2] for all i, j in [0, d), zero unless i1+i2 == j1+j2."""
    U = np.zeros((d, d, d, d), dtype=complex)
    for i1 in range(d):
        for i2 in range(d):
            for j1 in range(d):
                j2 = i1 + i2 - j1
                if 0 <= j2 < d:
                    U[i1, i2, j1, j2] = fock_amplitude(T, i1, i2, j1, j2)
    return U


def fock_block(T: np.ndarray, n: int) -> np.ndarray:
    """Full (n+1)x(n+1) block for total photon number n, [i1, j1] (no cutoff)."""
    B = np.zeros((n + 1, n + 1), dtype=complex)
    for i1 in range(n + 1):
        for j1 in range(n + 1):
            B[i1, j1] = fock_amplitude(T, i1, n - i1, j1, n - j1)
    return B
