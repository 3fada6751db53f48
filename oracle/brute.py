"""Full density-matrix evolution for tiny chains (oracle, FP64, M <= 4).

Test infrastructure only (see ``oracle/__init__``).

* rho = (x)_j rho_j (App. B, product input state after loss), stored as a
  tensor [m_1..m_M, m'_1..m'_M] over the per-mode cutoff [0, d).
* A beam splitter on modes (k, k+1) maps rho -> U rho U^dag with the two-mode
  Fock matrix restricted to the cutoff (Sec. II, unitary on a density
  operator).
* The U(1) operator entanglement entropy on bond b is computed by its
  definition: the vectorised state with the auxiliary total-charge leg is
  block diagonal in the charge q to the right of the bond (App. D), so its
  Schmidt values are the pooled singular values of the blocks
  rho[(left config), (right config of charge q)] over all q; the entropy is
  -sum p log2 p with p = lam^2 / sum lam^2 (Sec. II; App. B normalisation).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import fock


def product_rho(rhos):
    M = len(rhos)
    T = np.ones((), dtype=complex)
    for r in rhos:
        T = np.multiply.outer(T, r.astype(complex))      # appends (m, m')
    perm = [2 * i for i in range(M)] + [2 * i + 1 for i in range(M)]
    return np.transpose(T, perm)


def apply_gate(rho, m: int, theta: float, phi: float):
    """rho -> U rho U^dag for T(theta, phi) on modes (m, m+1)."""
    M = rho.ndim // 2
    d = rho.shape[0]
    Uf = fock.fock_bs(fock.bs_matrix(theta, phi), d)      # [I, J, i, j]
    # ket side
    rho = np.tensordot(Uf, rho, axes=([2, 3], [m, m + 1]))  # (I, J, rest...)
    rho = np.moveaxis(rho, [0, 1], [m, m + 1])
    # bra side: multiply by conj(U) on the bra indices
    rho = np.tensordot(Uf.conj(), rho, axes=([2, 3], [M + m, M + m + 1]))
    rho = np.moveaxis(rho, [0, 1], [M + m, M + m + 1])
    return rho


def apply_phases(rho, phases):
    M = rho.ndim // 2
    d = rho.shape[0]
    n = np.arange(d)
    for j, ph in enumerate(phases):
        shape = [1] * (2 * M)
        shape[j] = d
        rho = rho * np.exp(1j * ph * n).reshape(shape)
        shape = [1] * (2 * M)
        shape[M + j] = d
        rho = rho * np.exp(-1j * ph * n).reshape(shape)
    return rho


def u1_schmidt(rho, b: int):
    """Pooled Schmidt values with their right charges on bond b (0..M)."""
    M = rho.ndim // 2
    d = rho.shape[0]
    # vectorise with (m_j, m'_j) adjacent per mode
    perm = []
    for j in range(M):
        perm += [j, M + j]
    v = np.transpose(rho, perm)
    left = v.reshape(d ** (2 * b), d ** (2 * (M - b)))
    # right charge of every right configuration
    qs = {}
    for idx, cfg in enumerate(itertools.product(range(d), repeat=2 * (M - b))):
        q = (sum(cfg[0::2]), sum(cfg[1::2]))
        qs.setdefault(q, []).append(idx)
    vals, charges = [], []
    for q, cols in qs.items():
        s = np.linalg.svd(left[:, cols], compute_uv=False)
        vals.extend(s.tolist())
        charges.extend([q] * len(s))
    return np.array(vals), np.array(charges)


def u1_entropy(rho, b: int) -> float:
    s, _ = u1_schmidt(rho, b)
    p = s ** 2
    p = p / p.sum()
    p = p[p > 1e-300]
    return float(-(p * np.log2(p)).sum())


def marginals(rho):
    """(P[j, n] normalised, Tr rho)."""
    M = rho.ndim // 2
    d = rho.shape[0]
    diag = rho
    # take the diagonal of every mode
    for j in range(M):
        diag = np.diagonal(diag, axis1=0, axis2=M - j)   # moves diag axis to end
    # diag axes are now (m_1..m_M) in order
    P = np.zeros((M, d))
    for j in range(M):
        axes = tuple(a for a in range(M) if a != j)
        P[j] = diag.sum(axis=axes).real
    tr = float(diag.sum().real)
    return P / tr, tr
