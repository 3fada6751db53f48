"""Dense Vidal-form MPO of a lossy GBS state (oracle, FP64, no charge blocking).

Test infrastructure only (see ``oracle/__init__``).

Representation (Sec. II, Eq. MPS and the vectorisation map; App. D):
the vectorised density operator |rho>> = sum rho[k, k'] |k, k'> is written as

    Psi[alpha_0; (m_1, m'_1), ..., (m_M, m'_M)] =
        lam_0 G_0 lam_1 G_1 ... G_{M-1} lam_M

with site tensors G_j[a, m, m', b] (a on bond j, b on bond j+1, ket m, bra m')
and Schmidt values lam_b on bonds b = 0..M.  Bond 0 is an auxiliary left leg
whose index carries the total photon numbers (App. A: the charge of the
leftmost bond counts every photon); the physical state is the sum over that leg.
Charges c_b = (photons, photons') to the right of bond b (App. D) are carried
only as labels: every tensor here is dense and every contraction and SVD runs
on the full dense matrices.

Two-site update (App. D, Eq. Theta and the SVD that follows):
Theta = lam_{j} G_j lam_{j+1} G_{j+1} lam_{j+2}, the Fock beam splitter
U (x) conj(U) acts on the four local indices (Sec. II, vectorised unitary),
the dense SVD is truncated to chi, and G~_j = V / lam_j, G~_{j+1} = W^dag /
lam_{j+2}.

Truncation rule (the paper only says "keep the chi largest"; readings):
* singular values below 1e-14 of the largest are dropped (rank cut-off);
* Hermiticity makes the spectra of mirror charges (n, n') and (n', n)
  identical, so the i-th value of a sector and the i-th value of its mirror
  form one unit of size 2; a self-mirror sector gives units of size 1;
* units are taken by decreasing value (ties: canonical charge, then rank)
  while the running size stays <= chi; the first unit that does not fit ends
  the selection;
* the new bond is ordered by charge (lexicographic) then by decreasing value.
"""
from __future__ import annotations

import math

import numpy as np

from . import fock

RANK_CUT = 1e-14


# --------------------------------------------------------------------------
# truncation rule
# --------------------------------------------------------------------------
def select(charges: np.ndarray, vals: np.ndarray, chi: int) -> np.ndarray:
    """Indices kept by the mirror-pair rule, ordered by (charge, -value)."""
    vals = np.asarray(vals, dtype=float)
    if len(vals) == 0:
        return np.zeros(0, dtype=int)
    vmax = vals.max()
    groups: dict[tuple, list[int]] = {}
    for idx in range(len(vals)):
        if vals[idx] >= RANK_CUT * vmax and vals[idx] > 0:
            groups.setdefault((int(charges[idx][0]), int(charges[idx][1])), []).append(idx)
    for q in groups:
        groups[q].sort(key=lambda i: (-vals[i], i))
    units = []
    for q, members in groups.items():
        qb = (q[1], q[0])
        if q == qb:
            for i, idx in enumerate(members):
                units.append((vals[idx], q, i, [idx]))
        elif q < qb:
            partner = groups.get(qb, [])
            for i in range(max(len(members), len(partner))):
                mem = ([members[i]] if i < len(members) else []) + \
                      ([partner[i]] if i < len(partner) else [])
                units.append((max(vals[m] for m in mem), q, i, mem))
        elif qb not in groups:
            for i, idx in enumerate(members):
                units.append((vals[idx], qb, i, [idx]))
    units.sort(key=lambda u: (-u[0], u[1], u[2]))
    kept: list[int] = []
    for u in units:
        if len(kept) + len(u[3]) > chi:
            break
        kept.extend(u[3])
    kept.sort(key=lambda i: (int(charges[i][0]), int(charges[i][1]), -vals[i], i))
    return np.array(kept, dtype=int)


# --------------------------------------------------------------------------
# charge labels of dense singular vectors
# --------------------------------------------------------------------------
def _label_rows(Wh: np.ndarray, S: np.ndarray, col_charge: np.ndarray, V: np.ndarray):
    """Give every right singular vector (row of Wh) a definite charge.

    The dense SVD of a charge-block-diagonal matrix returns charge-definite
    vectors for non-degenerate values; inside a (near-)degenerate cluster it
    may return any rotation.  Inside each cluster the vectors are rotated to
    diagonalise the charge operator, which is exactly diagonal on the
    column basis.  Returns (labels, V, Wh) with V and Wh rotated consistently.
    """
    k = len(S)
    if k == 0:
        return np.zeros((0, 2), dtype=int), V, Wh
    keys = col_charge[:, 0].astype(np.int64) * 100003 + col_charge[:, 1].astype(np.int64)
    tol = 1e-11 * S[0]
    start = 0
    V = V.copy()
    Wh = Wh.copy()
    while start < k:
        end = start + 1
        while end < k and S[end - 1] - S[end] <= tol:
            end += 1
        if end - start > 1:
            blk = Wh[start:end]
            w = np.abs(blk) ** 2
            support = np.unique(keys[w.sum(axis=0) > 1e-12])
            f = np.zeros(len(keys))
            for rank, key in enumerate(support):
                f[keys == key] = rank + 1.0
            H = (blk * f[None, :]) @ blk.conj().T
            _, R = np.linalg.eigh(H)
            Wh[start:end] = R.conj().T @ blk
            V[:, start:end] = V[:, start:end] @ R
        start = end
    labels = np.zeros((k, 2), dtype=int)
    for i in range(k):
        w = np.abs(Wh[i]) ** 2
        tot = w.sum()
        uk, inv = np.unique(keys, return_inverse=True)
        acc = np.bincount(inv, weights=w, minlength=len(uk))
        best = int(np.argmax(acc))
        # a dense SVD resolves a vector's charge only up to rounding of the
        # largest value over the gap to its neighbours: for values near the
        # rank cut (far below 1e-8 of the largest) the leading charge is the label
        noisy = S[i] < 1e-8 * S[0] and acc[best] > 0.5 * tot
        if acc[best] < (1 - 1e-6) * tot and not noisy:
            raise RuntimeError("charge labelling failed: vector is not charge-definite")
        col = np.nonzero(inv == best)[0][0]
        labels[i] = col_charge[col]
    return labels, V, Wh


# --------------------------------------------------------------------------
# the MPO
# --------------------------------------------------------------------------
class DenseMPO:
    """Dense Vidal MPO with an auxiliary total-charge leg on bond 0."""

    def __init__(self, G, lam, charge, d):
        self.G = G            # list of M arrays (Dl, d, d, Dr), complex
        self.lam = lam        # list of M+1 real arrays
        self.charge = charge  # list of M+1 int arrays (D, 2)
        self.d = d

    @property
    def M(self):
        return len(self.G)

    # ---------------- initial state ----------------
    @classmethod
    def product(cls, rhos, chi: int, total_cap: int | None = None):
        """Initial state by its definition: the exact Vidal form of the product
        rho_1 (x) ... (x) rho_M with the auxiliary total-charge leg, written
        out from the Schmidt decomposition of a product state on every bond
        (one Schmidt vector per right charge q), then the top-chi
        (mirror-pair rule) charges kept on every bond without re-canonicalising.

        With w_b(q) the weight of charge q in (x)_{i>=b} rho_i (2-D
        convolution of |rho_i|^2) and V_b(q) the total weight of the left part
        (aux leg and modes i < b) that goes with right charge q:
        lam_b[q] = sqrt(w_b(q) V_b(q)) and
        G_j[q', m, m', q] = rho_j[m, m'] delta(q' = q + (m, m')) / (sqrt(V_{j+1}(q)) sqrt(w_j(q'))).
        Without a cap V_b(q) = prod_{i<b} ||rho_i||_F^2.  With ``total_cap``
        = K (App. A reading in which the cutoff bounds the total photon
        number: the aux charge, i.e. every photon, is at most K in ket and in
        bra), the state is projected onto totals <= K and V_b(q) is the left
        weight of charges p <= K - q.  ``product_by_sweeps`` obtains the same
        state by dense SVD sweeps.
        """
        M = len(rhos)
        d = rhos[0].shape[0]
        w = _weights(rhos)
        V = _left_weights(rhos, total_cap)
        bonds = product_bonds(rhos, chi, total_cap)
        charge = [bd[0] for bd in bonds]
        lam = [bd[1] for bd in bonds]
        G = []
        for j in range(M):
            idx = {tuple(q): i for i, q in enumerate(charge[j])}
            T = np.zeros((len(charge[j]), d, d, len(charge[j + 1])), dtype=complex)
            for qi, q in enumerate(charge[j + 1]):
                vq = V[j + 1](int(q[0]), int(q[1]))
                for m in range(d):
                    for mp in range(d):
                        key = (int(q[0]) + m, int(q[1]) + mp)
                        if rhos[j][m, mp] != 0 and key in idx:
                            a = idx[key]
                            T[a, m, mp, qi] = rhos[j][m, mp] / (math.sqrt(vq) *
                                                                math.sqrt(w[j][key]))
            G.append(T)
        return cls(G, lam, charge, d)

    @classmethod
    def product_by_sweeps(cls, rhos, chi: int, total_cap: int | None = None):
        """Vidal form of rho_1 (x) ... (x) rho_M by dense sweeps, then the top-chi
        (mirror-pair rule) charges kept on every bond, without re-canonicalising.
        Small sizes only: the dense SVD cannot resolve the vectors of Schmidt
        values far below the largest one.

        The charge-bond tensor B_j[q', m, m', q] = rho_j[m, m'] delta(q' = q + (m, m'))
        is the U(1) product MPO (App. D, the delta form of the MPS); the
        sweeps (QR left to right, SVD right to left) bring it to Vidal form
        exactly as for any MPS (App. D, Eq. MPS in Vidal form).  With
        ``total_cap`` = K the auxiliary leg keeps only totals <= K in ket and
        bra (projection of the state onto at most K photons).
        """
        M = len(rhos)
        d = rhos[0].shape[0]
        # reachable charges, counted from the right
        ch = [None] * (M + 1)
        ch[M] = [(0, 0)]
        for b in range(M - 1, -1, -1):
            s = set()
            nz = np.argwhere(rhos[b] != 0)
            for q in ch[b + 1]:
                for (m, mp) in nz:
                    s.add((q[0] + int(m), q[1] + int(mp)))
            ch[b] = sorted(s)
        if total_cap is not None:
            ch[0] = [q for q in ch[0] if q[0] <= total_cap and q[1] <= total_cap]
        index = [{q: i for i, q in enumerate(c)} for c in ch]
        B = []
        for j in range(M):
            T = np.zeros((len(ch[j]), d, d, len(ch[j + 1])), dtype=complex)
            for qi, q in enumerate(ch[j + 1]):
                for m in range(d):
                    for mp in range(d):
                        key = (q[0] + m, q[1] + mp)
                        if rhos[j][m, mp] != 0 and key in index[j]:
                            T[index[j][key], m, mp, qi] = rhos[j][m, mp]
            B.append(T)
        # left-canonicalise; bond 0 is an open leg (the auxiliary total charge)
        A = [t.copy() for t in B]
        for j in range(M - 1):
            Dl, _, _, Dr = A[j].shape
            Q, R = np.linalg.qr(A[j].reshape(Dl * d * d, Dr))
            A[j] = Q.reshape(Dl, d, d, Q.shape[1])
            A[j + 1] = np.tensordot(R, A[j + 1], axes=(1, 0))
        norm = np.linalg.norm(A[M - 1])
        lam = [None] * (M + 1)
        charge = [None] * (M + 1)
        Bright = [None] * M
        lam[M] = np.array([norm])
        charge[M] = np.array([[0, 0]])
        C = A[M - 1]
        aux_charge = np.array(ch[0])
        for j in range(M - 1, -1, -1):
            Dl, _, _, Dr = C.shape
            X = C.reshape(Dl, d * d * Dr)
            U_, S, Vh = np.linalg.svd(X, full_matrices=False)
            keep = S >= RANK_CUT * S[0]
            U_, S, Vh = U_[:, keep], S[keep], Vh[keep]
            col_charge = np.zeros((d, d, Dr, 2), dtype=int)
            for m in range(d):
                for mp in range(d):
                    col_charge[m, mp, :, 0] = charge[j + 1][:, 0] + m
                    col_charge[m, mp, :, 1] = charge[j + 1][:, 1] + mp
            labels, U_, Vh = _label_rows(Vh, S, col_charge.reshape(-1, 2), U_)
            Bright[j] = Vh.reshape(len(S), d, d, Dr)
            lam[j] = S
            charge[j] = labels
            if j > 0:
                C = np.tensordot(A[j - 1], U_ * S[None, :], axes=(3, 0))
            else:
                # bond 0: the left Schmidt vectors are aux basis states |Q>;
                # absorb their phases so that index alpha_0 is exactly |Q>.
                for a in range(len(S)):
                    qa = int(np.argmax(np.abs(U_[:, a])))
                    if abs(abs(U_[qa, a]) - 1) > 1e-8 or tuple(aux_charge[qa]) != tuple(labels[a]):
                        raise RuntimeError("bond-0 Schmidt vector is not an aux basis state")
                    Bright[0][a] *= U_[qa, a]
        G = []
        for j in range(M):
            G.append(Bright[j] / lam[j + 1][None, None, None, :])
        mpo = cls(G, lam, charge, d)
        mpo.truncate_all(chi)
        return mpo

    def truncate_all(self, chi: int):
        """Keep the top-chi (mirror-pair rule) indices on every bond, no
        re-canonicalisation (initial-state truncation)."""
        keep = [select(self.charge[b], self.lam[b], chi) for b in range(self.M + 1)]
        for b in range(self.M + 1):
            self.lam[b] = self.lam[b][keep[b]]
            self.charge[b] = self.charge[b][keep[b]]
        for j in range(self.M):
            self.G[j] = self.G[j][keep[j]][:, :, :, keep[j + 1]]

    # ---------------- gates ----------------
    def theta_matrix(self, m: int, theta: float, phi: float) -> np.ndarray:
        """Two-site tensor after the beam splitter T(theta, phi) on modes
        (m, m+1) (App. D, Eq. Theta; the vectorised unitary U (x) conj(U) of
        Sec. II on the (ket, bra) pairs of both modes), as the matrix
        X[(a, I, K), (J, L, b)] with I, K the ket / bra occupations of mode m
        and J, L those of mode m+1."""
        d = self.d
        j = m
        A, B = self.G[j], self.G[j + 1]
        lL, lC, lR = self.lam[j], self.lam[j + 1], self.lam[j + 2]
        Theta = np.einsum('a,aikc,c,cjlb,b->aikjlb', lL, A, lC, B, lR, optimize=True)
        Uf = fock.fock_bs(fock.bs_matrix(theta, phi), d)        # [I, J, i, j]
        # vectorised unitary U (x) conj(U) on (ket, bra) of both modes
        Theta = np.einsum('IJij,KLkl,aikjlb->aIKJLb', Uf, Uf.conj(), Theta, optimize=True)
        Dl, Dr = len(lL), len(lR)
        return Theta.reshape(Dl * d * d, d * d * Dr)

    def apply_gate(self, m: int, theta: float, phi: float, chi: int):
        """Beam splitter T(theta, phi) on modes (m, m+1): App. D two-site update."""
        d = self.d
        j = m
        lL, lR = self.lam[j], self.lam[j + 2]
        Dl, Dr = len(lL), len(lR)
        X = self.theta_matrix(m, theta, phi)
        V, S, Wh = np.linalg.svd(X, full_matrices=False)
        keep = S >= RANK_CUT * S[0] if len(S) and S[0] > 0 else np.zeros(len(S), bool)
        V, S, Wh = V[:, keep], S[keep], Wh[keep]
        col_charge = np.zeros((d, d, Dr, 2), dtype=int)
        cR = self.charge[j + 2]
        for J in range(d):
            for L in range(d):
                col_charge[J, L, :, 0] = cR[:, 0] + J
                col_charge[J, L, :, 1] = cR[:, 1] + L
        labels, V, Wh = _label_rows(Wh, S, col_charge.reshape(-1, 2), V)
        kept = select(labels, S, chi)
        S = S[kept]
        V = V[:, kept].reshape(Dl, d, d, len(kept))
        Wh = Wh[kept].reshape(len(kept), d, d, Dr)
        self.G[j] = V / lL[:, None, None, None]
        self.G[j + 1] = Wh / lR[None, None, None, :]
        self.lam[j + 1] = S
        self.charge[j + 1] = labels[kept]

    def apply_phases(self, phases):
        """Output phase screen D: |n> -> e^{i n phi}|n> on every mode, i.e.
        rho[m, m'] -> e^{i phi (m - m')} rho[m, m'] (Sec. II, vectorised unitary)."""
        d = self.d
        n = np.arange(d)
        for j, ph in enumerate(phases):
            f = np.exp(1j * ph * (n[:, None] - n[None, :]))
            self.G[j] = self.G[j] * f[None, :, :, None]

    # ---------------- readouts ----------------
    def entropies(self):
        """Operator EE on bonds 1..M-1, in bits, with p = lam^2 / sum lam^2
        (Sec. II EE definition; App. B normalisation and log base 2)."""
        out = []
        for b in range(1, self.M):
            p = self.lam[b] ** 2
            p = p / p.sum()
            p = p[p > 0]
            out.append(float(-(p * np.log2(p)).sum()))
        return np.array(out)

    def renyi(self, alpha: float):
        """Renyi-alpha operator entropies on bonds 1..M-1, in bits, of the same
        normalised spectra p = lam^2 / sum lam^2 (Sec. III.B, App. B):
        log2(sum p^alpha) / (1 - alpha); alpha = 1 is the EE above."""
        out = []
        for b in range(1, self.M):
            p = self.lam[b] ** 2
            p = p / p.sum()
            p = p[p > 0]
            if alpha == 1.0:
                out.append(float(-(p * np.log2(p)).sum()))
            else:
                out.append(float(math.log2((p ** alpha).sum()) / (1.0 - alpha)))
        return np.array(out)

    def marginals(self):
        """(P[j, n] = Tr(rho Pi_{j,n}) / Tr rho, Tr rho, raw Tr(rho Pi)).

        The trace contracts every site with the identity (local m = m') and
        the auxiliary leg with the all-ones vector; 1 - Tr rho is the paper's
        error proxy (Sec. I, Sec. III, App. A)."""
        M, d = self.M, self.d
        diag = [np.einsum('ammb->amb', g) for g in self.G]     # (Dl, d, Dr)
        E = [None] * (M + 1)
        E[M] = np.ones(1, dtype=complex)
        for j in range(M - 1, -1, -1):
            E[j] = np.einsum('amb,b,b->a', diag[j], self.lam[j + 1], E[j + 1])
        L = [None] * (M + 1)
        L[0] = np.ones(len(self.lam[0]), dtype=complex)
        for j in range(M):
            L[j + 1] = np.einsum('a,a,amb->b', L[j], self.lam[j], diag[j])
        raw = np.zeros((M, d))
        for j in range(M):
            v = np.einsum('a,a,amb,b,b->m', L[j], self.lam[j], diag[j],
                          self.lam[j + 1], E[j + 1])
            raw[j] = v.real
        tr = float(np.sum(L[0] * self.lam[0] * E[0]).real)
        return raw / tr, tr, raw

    def to_dense(self):
        """Full rho as a tensor [m_1..m_M, m'_1..m'_M] (sums the aux leg)."""
        M, d = self.M, self.d
        T = np.diag(self.lam[0]).astype(complex)   # (aux, bond 0)
        for j in range(M):
            g = self.G[j] * self.lam[j + 1][None, None, None, :]
            T = np.tensordot(T, g, axes=(T.ndim - 1, 0))
        T = T.sum(axis=0)                          # sum over the aux leg
        T = T[..., 0]                              # bond M has one index
        perm = [2 * i for i in range(M)] + [2 * i + 1 for i in range(M)]
        return np.transpose(T, perm)


def _weights(rhos):
    """w_b on the grid [0, (M-b)(d-1)]^2: 2-D convolution of |rho_j|^2, j >= b."""
    M = len(rhos)
    d = rhos[0].shape[0]
    w = [None] * (M + 1)
    w[M] = np.ones((1, 1))
    for b in range(M - 1, -1, -1):
        prev = w[b + 1]
        W = prev.shape[0] + d - 1
        acc = np.zeros((W, W))
        a2 = np.abs(rhos[b]) ** 2
        for m in range(d):
            for mp in range(d):
                if a2[m, mp] != 0:
                    acc[m:m + prev.shape[0], mp:mp + prev.shape[1]] += a2[m, mp] * prev
        w[b] = acc
    return w


def _left_weights(rhos, total_cap):
    """Per bond b a function V_b(q): the squared norm of the left part that
    goes with right charge q.  Without a cap it is prod_{j<b} ||rho_j||_F^2.
    With a total cap K the aux charge Q = p + q (p = photons of modes j < b)
    must stay <= K, so V_b(q) = sum_{p <= K - q} u_b(p), u_b the 2-D
    convolution of |rho_j|^2 over j < b (u_0 = delta_0); 0 if q exceeds K."""
    M = len(rhos)
    if total_cap is None:
        out, A2 = [], 1.0
        for b in range(M + 1):
            out.append(lambda q0, q1, A2=A2: A2)
            if b < M:
                A2 *= float((np.abs(rhos[b]) ** 2).sum())
        return out
    K = total_cap
    d = rhos[0].shape[0]
    u = np.zeros((K + 1, K + 1))
    u[0, 0] = 1.0
    out = []
    for b in range(M + 1):
        cum = np.cumsum(np.cumsum(u, axis=0), axis=1)
        out.append(lambda q0, q1, cum=cum: float(cum[K - q0, K - q1])
                   if 0 <= q0 <= K and 0 <= q1 <= K else 0.0)
        if b < M:
            nu = np.zeros_like(u)
            a2 = np.abs(rhos[b]) ** 2
            for m in range(min(d, K + 1)):
                for mp in range(min(d, K + 1)):
                    nu[m:, mp:] += a2[m, mp] * u[: K + 1 - m, : K + 1 - mp]
            u = nu
    return out


def product_lambdas(rhos, total_cap: int | None = None):
    """Closed form of the untruncated product-state Schmidt values with the
    auxiliary leg: lam_b[q]^2 = w_b(q) V_b(q), w_b the 2-D convolution of
    |rho_j|^2 over modes j >= b and V_b the left weight (``_left_weights``;
    App. D charges: the Schmidt decomposition of a product state has one
    vector per right charge).  Returns per bond a dict {q: lam} over the
    charges with a positive value."""
    M = len(rhos)
    w = _weights(rhos)
    V = _left_weights(rhos, total_cap)
    out = []
    for b in range(M + 1):
        nz = np.argwhere(w[b] > 0)
        vals = {(int(q0), int(q1)): math.sqrt(V[b](int(q0), int(q1)) * w[b][q0, q1])
                for q0, q1 in nz}
        out.append({q: v for q, v in vals.items() if v > 0})
    return out


def product_bonds(rhos, chi: int, total_cap: int | None = None):
    """Bond charges and Schmidt values of the initial state after the top-chi
    (mirror-pair rule) truncation of every bond, without building tensors."""
    lam_d = product_lambdas(rhos, total_cap)
    out = []
    for ld in lam_d:
        ch = np.array(sorted(ld.keys()), dtype=int).reshape(-1, 2)
        lam = np.array([ld[tuple(q)] for q in ch])
        keep = select(ch, lam, chi)
        out.append((ch[keep], lam[keep]))
    return out


# --------------------------------------------------------------------------
# one charge sector of the two-site tensor, in the charge-blocked form
# --------------------------------------------------------------------------
def sector_theta(Gj, Gj1, lamL, lamC, lamR, cL, cC, cR, theta: float, phi: float, d: int, q):
    """Charge sector q of the two-site tensor after a beam splitter, from the
    charge-blocked Vidal form (App. D, Eq. Theta restricted to one new centre
    charge; beam splitter as in Sec. II).

    In the blocked form a site is a bond-by-bond matrix, Gj[a, alpha], whose
    local (ket, bra) occupations are fixed by the charges: m = c_a - c_alpha.
    With p = c_alpha and n = c_a - c_b,
        Theta(q)[a, b] = lamL[a] lamR[b] sum_alpha Gj[a, alpha] lamC[alpha] Gj1[alpha, b]
                         U[c_a0 - q0, q0 - c_b0, c_a0 - p0, p0 - c_b0]
                         conj(U[c_a1 - q1, q1 - c_b1, c_a1 - p1, p1 - c_b1])
    where U[I, J, i, j] is the two-mode Fock matrix (outputs I, J, inputs
    i, j) and every occupation lies in [0, d).  Rows are the left-bond
    indices a with c_a - q in [0, d)^2, columns the right-bond indices b
    with q - c_b in [0, d)^2.  Returns (rows, cols, Theta(q)).

    Slow and direct: one matrix product per centre charge p (no blocking
    beyond the charge grouping the definition implies).
    """
    Uf = fock.fock_bs(fock.bs_matrix(theta, phi), d)
    cL, cC, cR = np.asarray(cL), np.asarray(cC), np.asarray(cR)
    q = np.asarray(q)

    def inside(x):
        return np.all((x >= 0) & (x < d), axis=-1)

    rows = np.nonzero(inside(cL - q))[0]
    cols = np.nonzero(inside(q - cR))[0]
    Th = np.zeros((len(rows), len(cols)), dtype=complex)
    if len(rows) == 0 or len(cols) == 0:
        return rows, cols, Th
    ca = cL[rows]                      # (r, 2)
    cb = cR[cols]                      # (s, 2)
    for p in np.unique(cC, axis=0):
        # the delta factors of Eq. theta admit a term only on the rows whose
        # old occupation c_a - p and the columns whose c_b side p - c_b lie in
        # the cutoff; the term is evaluated on that sub-block alone
        ri = np.nonzero(inside(ca - p))[0]
        ci = np.nonzero(inside(p - cb))[0]
        if len(ri) == 0 or len(ci) == 0:
            continue
        al = np.nonzero(np.all(cC == p, axis=1))[0]
        Gp = (Gj[np.ix_(rows[ri], al)] * lamC[al][None, :]) @ Gj1[np.ix_(al, cols[ci])]
        a_ = ca[ri][:, None, :]         # (r', 1, 2)
        b_ = cb[ci][None, :, :]         # (1, s', 2)
        I_out = np.broadcast_to(a_ - q, (len(ri), len(ci), 2))
        J_out = np.broadcast_to(q - b_, (len(ri), len(ci), 2))
        i_in = np.broadcast_to(a_ - p, (len(ri), len(ci), 2))   # mode m before the gate
        j_in = np.broadcast_to(p - b_, (len(ri), len(ci), 2))   # mode m+1 before the gate
        ket = Uf[I_out[..., 0], J_out[..., 0], i_in[..., 0], j_in[..., 0]]
        bra = Uf[I_out[..., 1], J_out[..., 1], i_in[..., 1], j_in[..., 1]]
        Th[np.ix_(ri, ci)] += ket * np.conj(bra) * Gp
    return rows, cols, Th * lamL[rows][:, None] * lamR[cols][None, :]
