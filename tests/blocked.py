"""Test helpers that read the library's charge-blocked Vidal form back into
dense objects (test infrastructure; written from the representation, shares
no code with the library or the oracle).

In the blocked form (App. D) a site is a bond-by-bond matrix Gamma_j[a, b]
whose local (ket, bra) occupation is fixed by the right-counted charges:
(m, m') = c_j[a] - c_{j+1}[b].  The state is
    rho[m_1..m_M; m'_1..m'_M] = sum lam_0 Gamma_0 lam_1 Gamma_1 ... Gamma_{M-1} lam_M
with the auxiliary leg (bond 0) summed over.
"""
from __future__ import annotations

import numpy as np


def expand_site(G, cl, cr, d):
    """Gamma_j[a, b] -> dense T[a, m, m', b]; also returns the largest |entry|
    found outside the charge-compatible pattern (which must be zero)."""
    Dl, Dr = G.shape
    T = np.zeros((Dl, d, d, Dr), dtype=complex)
    diff = cl[:, None, :] - cr[None, :, :]                  # (Dl, Dr, 2)
    ok = np.all((diff >= 0) & (diff < d), axis=-1)
    a, b = np.nonzero(ok)
    T[a, diff[a, b, 0], diff[a, b, 1], b] = G[a, b]
    outside = float(np.abs(G[~ok]).max()) if (~ok).any() else 0.0
    return T, outside


def library_rho(g, M, d):
    """Full density matrix [m_1..m_M, m'_1..m'_M] of a library MPO handle, and
    the largest Gamma entry outside the charge pattern."""
    bonds = [g.bond(b) for b in range(M + 1)]
    T = bonds[0][0].astype(complex)                          # sum over the aux leg
    worst = 0.0
    for j in range(M):
        S, out = expand_site(g.site(j), bonds[j][1], bonds[j + 1][1], d)
        worst = max(worst, out)
        S = S * bonds[j + 1][0][None, None, None, :]
        T = np.tensordot(T, S, axes=(T.ndim - 1, 0))
    T = T[..., 0]                                            # bond M has one index
    perm = [2 * i for i in range(M)] + [2 * i + 1 for i in range(M)]
    return np.transpose(T, perm), worst
