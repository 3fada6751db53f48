"""Interferometer -> rectangular mesh of nearest-neighbour beam splitters (oracle).

Test infrastructure only (see ``oracle/__init__``).

The paper builds its global Haar-random interferometers as an M-layer array
(App. A).  This module writes the rectangular decomposition of Clements et al.
(Optica 3, 1460 (2016)): M(M-1)/2 beam splitters T(theta, phi) on
neighbouring modes, whose ASAP layering has depth M, followed by a diagonal
phase screen D.  Conventions:

* T(theta, phi) = [[e^{i phi} cos t, -sin t], [e^{i phi} sin t, cos t]] acting
  on modes (m, m+1); a^dag_j -> sum_i U[i, j] a^dag_i, so a sequence of
  elements T_1, T_2, ... composes to U = D ... T_2 T_1.
* theta in [0, pi/2], phi in (-pi, pi].

Returned gates are in application order.
"""
from __future__ import annotations

import math

import numpy as np


def _embed(M: int, m: int, T: np.ndarray) -> np.ndarray:
    E = np.eye(M, dtype=complex)
    E[m:m + 2, m:m + 2] = T
    return E


def _T(theta: float, phi: float) -> np.ndarray:
    e = np.exp(1j * phi)
    return np.array([[e * math.cos(theta), -math.sin(theta)],
                     [e * math.sin(theta), math.cos(theta)]], dtype=complex)


def _wrap(phi: float) -> float:
    """Map an angle to (-pi, pi]."""
    x = math.remainder(phi, 2 * math.pi)
    return math.pi if x == -math.pi else x


def decompose(U: np.ndarray):
    """Return (gates, phases): gates = [(m, theta, phi), ...] in application
    order, phases = arg of the diagonal screen D, with U = D * prod(T)."""
    M = U.shape[0]
    V = np.array(U, dtype=complex)
    right = []   # V <- V @ T^dag on columns (m, m+1)
    left = []    # V <- T @ V on rows (m, m+1)
    for i in range(M - 1):
        if i % 2 == 0:
            for j in range(i + 1):
                row, col = M - 1 - j, i - j
                a, b = V[row, col], V[row, col + 1]
                theta = math.atan2(abs(a), abs(b))
                phi = 0.0 if (a == 0 or b == 0) else _wrap(np.angle(a) - np.angle(b))
                V = V @ _embed(M, col, _T(theta, phi)).conj().T
                right.append((col, theta, phi))
        else:
            for j in range(i + 1):
                row, col = M - 1 - i + j, j
                a, b = V[row - 1, col], V[row, col]
                theta = math.atan2(abs(b), abs(a))
                phi = 0.0 if (a == 0 or b == 0) else _wrap(math.pi + np.angle(b) - np.angle(a))
                V = _embed(M, row - 1, _T(theta, phi)) @ V
                left.append((row - 1, theta, phi))
    diag = np.diag(V).copy()
    # Move every left element through the diagonal: L^dag D = D' T(theta, phi')
    # with phi' = arg(-d_m / d_{m+1}), d'_m = -e^{-i phi} d_{m+1}, d'_{m+1} = d_{m+1}.
    moved = []
    for (m, theta, phi) in reversed(left):
        d1, d2 = diag[m], diag[m + 1]
        phi_new = _wrap(np.angle(-d1 / d2))
        diag[m] = -np.exp(-1j * phi) * d2
        moved.append((m, theta, phi_new))
    gates = right + moved
    phases = np.angle(diag)
    return gates, phases


def reconstruct(M: int, gates, phases) -> np.ndarray:
    """U = D * T_L * ... * T_1 from the application-ordered gate list."""
    U = np.eye(M, dtype=complex)
    for (m, theta, phi) in gates:
        U = _embed(M, m, _T(theta, phi)) @ U
    return np.diag(np.exp(1j * np.asarray(phases))) @ U


def layers(M: int, gates):
    """Greedy as-soon-as-possible layering into sets of disjoint pairs."""
    last = [0] * M
    out: list[list[tuple]] = []
    for g in gates:
        m = g[0]
        L = max(last[m], last[m + 1])
        if L == len(out):
            out.append([])
        out[L].append(g)
        last[m] = last[m + 1] = L + 1
    return out
