"""Pins of the oracle's dense Vidal MPO (Sec. II; App. D) against brute-force
density-matrix evolution, closed forms and invariants."""
import itertools
import math

import numpy as np
import pytest

from oracle import brute, clements, fock, mpo, states
from paper_2301_12814_amd import inputs
from tests import closed_forms as cf


def _rhos(M, d, r, eta):
    r = r if isinstance(r, (list, tuple)) else [r] * M
    return [states.lossy_squeezed_rho(rj, eta, d) for rj in r]


def _bond_charges(M, d):
    """charge at bond b of every configuration (ket tuple, bra tuple)."""
    out = {}
    for ket in itertools.product(range(d), repeat=M):
        for bra in itertools.product(range(d), repeat=M):
            out[(ket, bra)] = [(sum(ket[b:]), sum(bra[b:])) for b in range(M + 1)]
    return out


def _sorted_desc(x):
    return np.sort(np.asarray(x))[::-1]


# ------------------------------------------------------------------ selection
def test_select_pairs_and_stop_rule():
    ch = np.array([[0, 2], [2, 0], [1, 1], [3, 1], [1, 3], [2, 2]])
    v = np.array([0.9, 0.9, 0.8, 0.7, 0.7, 0.6])
    assert list(mpo.select(ch, v, 6)) == [0, 2, 4, 1, 5, 3]     # ordered by charge
    # chi = 4: (0,2)+(2,0) [2], (1,1) [1], then the (1,3)/(3,1) pair does not fit
    kept = mpo.select(ch, v, 4)
    assert sorted(kept.tolist()) == [0, 1, 2]
    # rank cut-off 1e-14 relative
    v2 = np.array([1.0, 1.0, 1e-15, 0.5, 0.5, 0.0])
    assert sorted(mpo.select(ch, v2, 10).tolist()) == [0, 1, 3, 4]
    # within a charge, decreasing value
    ch3 = np.array([[1, 1], [1, 1], [1, 1]])
    assert list(mpo.select(ch3, np.array([0.1, 0.3, 0.2]), 2)) == [1, 2]


# ------------------------------------------------------------------ initial state
@pytest.mark.parametrize("M,d,r,eta", [(3, 4, 0.5, 0.5), (4, 3, [0.9, 0.0, 0.4, 0.7], 0.6)])
def test_product_init_matches_brute_force_and_closed_form(M, d, r, eta):
    rhos = _rhos(M, d, r, eta)
    m = mpo.DenseMPO.product_by_sweeps(rhos, 10 ** 6)
    mc = mpo.DenseMPO.product(rhos, 10 ** 6)
    rho = brute.product_rho(rhos)
    assert np.abs(m.to_dense() - rho).max() < 1e-14
    assert np.abs(mc.to_dense() - rho).max() < 1e-14
    for b in range(M + 1):
        assert np.array_equal(mc.charge[b], m.charge[b])
        assert np.allclose(mc.lam[b], m.lam[b], rtol=1e-12)
    closed = mpo.product_lambdas(rhos)
    for b in range(M + 1):
        s, c = brute.u1_schmidt(rho, b)
        keep = s >= 1e-14 * s.max()
        assert np.allclose(_sorted_desc(m.lam[b]), _sorted_desc(s[keep]), rtol=1e-12, atol=1e-15)
        for q, lam in zip(m.charge[b], m.lam[b]):
            assert abs(closed[b][tuple(q)] - lam) <= 1e-12 * lam
    # product state: U(1) EE > 0 while the plain operator EE is 0 (Sec. III.C remark)
    S = m.entropies()
    assert np.all(S[np.array([len(l) for l in m.lam[1:M]]) > 1] > 0.01)
    perm = []
    for j in range(M):
        perm += [j, M + j]
    vec = np.transpose(rho, perm).reshape(d ** 2, -1)
    sv = np.linalg.svd(vec, compute_uv=False)
    assert sv[1] < 1e-14 * sv[0]


def test_init_truncation_is_projection_onto_kept_charges():
    M, d, chi = 4, 3, 7
    rhos = _rhos(M, d, 0.8, 0.7)
    m = mpo.DenseMPO.product(rhos, chi)
    full = mpo.DenseMPO.product(rhos, 10 ** 6)
    rho = brute.product_rho(rhos)
    kept = [set(map(tuple, m.charge[b])) for b in range(M + 1)]
    ref = rho.copy()
    for (ket, bra), qs in _bond_charges(M, d).items():
        if not all(qs[b] in kept[b] for b in range(M + 1)):
            ref[ket + bra] = 0
    assert np.abs(m.to_dense() - ref).max() < 1e-14
    for b in range(M + 1):
        assert len(m.lam[b]) <= chi
        allv = full.lam[b]
        if len(allv) > chi:
            assert len(m.lam[b]) >= chi - 1
        dropped = sorted(set(map(tuple, full.charge[b])) - kept[b])
        if dropped:
            dv = max(full.lam[b][i] for i in range(len(allv)) if tuple(full.charge[b][i]) in dropped)
            assert dv <= m.lam[b].min() * (1 + 1e-12)
        assert kept[b] == {(q[1], q[0]) for q in kept[b]}          # mirror closed


def test_initial_trace_is_product_of_cropped_traces():
    M, d = 4, 3
    r = [0.9, 0.2, 0.0, 0.6]
    rhos = _rhos(M, d, r, 0.45)
    m = mpo.DenseMPO.product(rhos, 10 ** 6)
    _, tr, _ = m.marginals()
    ref = np.prod([np.trace(x) for x in rhos])
    assert abs(tr - ref) < 1e-14
    for j in range(M):
        P, _, _ = m.marginals()
        assert np.abs(P[j] - np.diag(rhos[j]) / np.trace(rhos[j])).max() < 1e-14


# ------------------------------------------------------------------ gates
@pytest.mark.parametrize("M,d,seed", [(3, 4, 11), (4, 3, 12)])
def test_gates_match_brute_force(M, d, seed):
    rhos = _rhos(M, d, [0.7, 0.4, 0.9, 0.3][:M], 0.6)
    U = inputs.haar_unitary(M, seed)
    gates, phases = clements.decompose(U)
    m = mpo.DenseMPO.product(rhos, 10 ** 6)
    rho = brute.product_rho(rhos)
    for (k, th, ph) in gates:
        m.apply_gate(k, th, ph, 10 ** 6)
        rho = brute.apply_gate(rho, k, th, ph)
        dense = m.to_dense()
        assert np.abs(dense - rho).max() < 1e-13
        # the updated bond carries exact Schmidt values of the new state when
        # its left basis is still orthonormal (always for the first bond)
        if k == 0:
            s, c = brute.u1_schmidt(rho, 1)
            s = s[s >= 1e-14 * s.max()]
            assert np.allclose(_sorted_desc(m.lam[1]), _sorted_desc(s), rtol=1e-10, atol=1e-14)
    m.apply_phases(phases)
    rho = brute.apply_phases(rho, phases)
    dense = m.to_dense()
    assert np.abs(dense - rho).max() < 1e-13
    n = rho.ndim // 2
    mat = rho.reshape(d ** n, d ** n)
    assert np.abs(mat - mat.conj().T).max() < 1e-15            # rho = rho^dag
    P, tr, _ = m.marginals()
    P2, tr2 = brute.marginals(rho)
    assert abs(tr - tr2) < 1e-13 and np.abs(P - P2).max() < 1e-13


def _bounded_rhos(M, d, seed):
    """Mixed states with at most one photon per mode (ket and bra), any phases."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(M):
        X = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        r2 = X @ X.conj().T
        r2 /= np.trace(r2).real
        R = np.zeros((d, d), dtype=complex)
        R[:2, :2] = r2
        out.append(R)
    return out


def test_every_bond_exact_without_leakage():
    """With total photons below the cutoff the restricted beam splitter is
    unitary on the support, the Vidal form stays exact and every bond's
    Schmidt values and U(1) EE equal the brute-force ones."""
    M, d = 3, 4
    rhos = _bounded_rhos(M, d, 3)
    U = inputs.haar_unitary(M, 4)
    gates, _ = clements.decompose(U)
    m = mpo.DenseMPO.product(rhos, 10 ** 6)
    rho = brute.product_rho(rhos)
    for (k, th, ph) in gates:
        m.apply_gate(k, th, ph, 10 ** 6)
        rho = brute.apply_gate(rho, k, th, ph)
        for b in range(M + 1):
            s, _ = brute.u1_schmidt(rho, b)
            s = s[s >= 1e-14 * s.max()]
            assert np.allclose(_sorted_desc(m.lam[b]), _sorted_desc(s), rtol=1e-10, atol=1e-14)
        Sm = m.entropies()
        for b in range(1, M):
            assert abs(Sm[b - 1] - brute.u1_entropy(rho, b)) < 1e-10
        _, tr, _ = m.marginals()
        assert abs(tr - 1) < 1e-13                              # no leak


def test_gate_truncation_keeps_top_schmidt_components():
    M, d, chi = 3, 4, 12
    rhos = _rhos(M, d, [0.9, 0.8, 0.7], 0.7)
    m = mpo.DenseMPO.product(rhos, 10 ** 6)
    rho = brute.product_rho(rhos)
    th, ph = 0.6, 0.4
    m.apply_gate(0, th, ph, chi)
    rho = brute.apply_gate(rho, 0, th, ph)
    # brute-force Schmidt decomposition on bond 1 by right charge
    perm = []
    for j in range(M):
        perm += [j, M + j]
    v = np.transpose(rho, perm)
    left = v.reshape(d ** 2, d ** 4)
    cfgs = list(itertools.product(range(d), repeat=4))
    groups = {}
    for idx, cfg in enumerate(cfgs):
        groups.setdefault((cfg[0] + cfg[2], cfg[1] + cfg[3]), []).append(idx)
    counts = {}
    for q in map(tuple, m.charge[1]):
        counts[q] = counts.get(q, 0) + 1
    approx = np.zeros_like(left)
    all_vals, kept_vals = [], []
    for q, cols in groups.items():
        u, s, vh = np.linalg.svd(left[:, cols], full_matrices=False)
        k = counts.get(q, 0)
        approx[:, cols] = (u[:, :k] * s[:k]) @ vh[:k]
        all_vals += [(x, q) for x in s if x > 1e-14]
        kept_vals += list(s[:k])
        mine = np.sort(m.lam[1][[tuple(c) == q for c in m.charge[1]]])[::-1]
        assert np.allclose(mine, s[:k], rtol=1e-10)
    dense = np.transpose(m.to_dense(), perm).reshape(d ** 2, d ** 4)
    assert np.abs(dense - approx).max() < 1e-13
    assert len(kept_vals) in (chi - 1, chi)
    dropped = sorted([x for x, _ in all_vals], reverse=True)[len(kept_vals):]
    assert max(dropped) <= min(kept_vals) * (1 + 1e-10)


def test_truncated_run_is_hermitian_and_mirror_symmetric():
    w = inputs.Workload("t", 5, [0.6] * 5, 0.5, 3, 10, 9)
    rhos = _rhos(w.M, w.d, w.r, w.eta)
    U = inputs.haar_unitary(w.M, w.seed)
    gates, phases = clements.decompose(U)
    m = mpo.DenseMPO.product(rhos, w.chi)
    for (k, th, ph) in gates:
        m.apply_gate(k, th, ph, w.chi)
        for b in range(w.M + 1):
            byq = {}
            for q, l in zip(map(tuple, m.charge[b]), m.lam[b]):
                byq.setdefault(q, []).append(l)
            for q, ls in byq.items():
                mir = byq[(q[1], q[0])]
                assert np.allclose(sorted(ls), sorted(mir), rtol=1e-10)
    n = w.M
    mat = m.to_dense().reshape(w.d ** n, w.d ** n)
    assert np.abs(mat - mat.conj().T).max() < 1e-14


# ------------------------------------------------------------------ closed forms
def test_marginals_match_gaussian_closed_form():
    """Output photon statistics of a lossy squeezed two-mode interferometer,
    exact as d -> infinity; at d = 10 the gap is bounded by the leaked mass."""
    M, d, r, eta = 2, 10, [0.5, 0.35], 0.5
    rhos = _rhos(M, d, r, eta)
    U = inputs.haar_unitary(M, 21)
    gates, phases = clements.decompose(U)
    m = mpo.DenseMPO.product(rhos, 10 ** 6)
    for (k, th, ph) in gates:
        m.apply_gate(k, th, ph, 10 ** 6)
    m.apply_phases(phases)
    P, tr, raw = m.marginals()
    N, A = cf.output_mode_moments(U, r, eta)
    leak = 1 - tr
    assert 0 <= leak < 1e-5
    for i in range(M):
        Pc = cf.gaussian_photon_distribution(N[i], A[i], d)
        assert np.abs(raw[i] - Pc).max() <= leak + 1e-12
    # mean photon number is conserved up to the leaked mass
    n = np.arange(d)
    mean_out = sum((n * raw[i]).sum() for i in range(M))
    assert abs(mean_out - eta * sum(math.sinh(x) ** 2 for x in r)) < 2 * d * leak + 1e-10


def test_special_cases():
    M, d = 3, 3
    rhos = _rhos(M, d, 0.7, 0.6)
    m = mpo.DenseMPO.product(rhos, 10 ** 6)
    lam0 = [l.copy() for l in m.lam]
    ch0 = [c.copy() for c in m.charge]
    S0 = m.entropies()
    P0, tr0, _ = m.marginals()
    m.apply_gate(1, 0.0, 0.0, 10 ** 6)                      # identity
    for b in range(M + 1):
        assert np.array_equal(m.charge[b], ch0[b])
        assert np.allclose(m.lam[b], lam0[b], rtol=1e-13)
    m.apply_gate(0, 0.0, 1.3, 10 ** 6)                      # phases only
    m.apply_phases([0.3, -1.0, 2.0])
    assert np.allclose(m.entropies(), S0, atol=1e-12)
    P1, tr1, _ = m.marginals()
    assert np.abs(P1 - P0).max() < 1e-13 and abs(tr1 - tr0) < 1e-13
    # all-vacuum input: one charge (0, 0), EE 0, P = delta_{n0}
    vac = _rhos(M, d, 0.0, 0.5)
    m = mpo.DenseMPO.product(vac, 8)
    for (k, th, ph) in [(0, 0.4, 0.1), (1, 0.9, 2.0)]:
        m.apply_gate(k, th, ph, 8)
    assert all(len(l) == 1 and tuple(c[0]) == (0, 0) for l, c in zip(m.lam, m.charge))
    assert np.allclose(m.entropies(), 0)
    P, tr, _ = m.marginals()
    assert abs(tr - 1) < 1e-15 and np.allclose(P[:, 0], 1) and np.allclose(P[:, 1:], 0)


# ------------------------------------------------------- charge-sector Theta
def _blocked_sites(o, j):
    """Charge-blocked site matrix Gj[a, alpha] of the dense site tensor
    G[a, m, m', alpha]: the entry at the occupations the charges fix."""
    G = o.G[j]
    cL, cR = o.charge[j], o.charge[j + 1]
    d = o.d
    out = np.zeros((G.shape[0], G.shape[3]), dtype=complex)
    for a in range(G.shape[0]):
        for al in range(G.shape[3]):
            m0, m1 = cL[a] - cR[al]
            if 0 <= m0 < d and 0 <= m1 < d:
                out[a, al] = G[a, m0, m1, al]
    return out


@pytest.mark.parametrize("M,d,chi,seed", [(5, 4, 24, 3), (4, 5, 40, 4)])
def test_sector_theta_matches_dense_theta(M, d, chi, seed):
    """Every charge sector of the blocked two-site tensor equals the rows
    (a, c_a - q) and columns (q - c_b, b) of the dense tensor after the gate,
    on a state that earlier gates have entangled."""
    rng = np.random.default_rng(seed)
    o = mpo.DenseMPO.product(_rhos(M, d, [0.8, 0.5, 0.9, 0.6, 0.7][:M], 0.6), chi)
    for k in (0, 2, 1):
        if k + 1 < M:
            o.apply_gate(k, float(rng.uniform(0, 1.5)), float(rng.uniform(-3, 3)), chi)
    j = 1
    th, ph = 0.83, -1.2
    X = o.theta_matrix(j, th, ph)
    cL, cC, cR = o.charge[j], o.charge[j + 1], o.charge[j + 2]
    Gj, Gj1 = _blocked_sites(o, j), _blocked_sites(o, j + 1)
    Dr = len(cR)
    qs = {tuple(int(x) for x in cL[a] - np.array([i, k]))
          for a in range(len(cL)) for i in range(d) for k in range(d)}
    scale = np.abs(X).max()
    seen = 0
    covered = np.zeros(X.shape, dtype=bool)
    for q in sorted(qs):
        rows, cols, Th = mpo.sector_theta(Gj, Gj1, o.lam[j], o.lam[j + 1], o.lam[j + 2],
                                          cL, cC, cR, th, ph, d, q)
        if len(rows) == 0 or len(cols) == 0:
            continue
        ri = [(a * d + (cL[a][0] - q[0])) * d + (cL[a][1] - q[1]) for a in rows]
        ci = [((q[0] - cR[b][0]) * d + (q[1] - cR[b][1])) * Dr + b for b in cols]
        assert np.abs(X[np.ix_(ri, ci)] - Th).max() <= 1e-12 * scale, q
        covered[np.ix_(ri, ci)] = True
        seen += 1
    assert seen > 5
    # the sectors hold the whole tensor: nothing outside them
    assert np.abs(X[~covered]).max() <= 1e-12 * scale


def test_renyi_entropies_against_charge_resolved_purity():
    """Renyi readout of the dense MPO (Sec. III.B): alpha = 2 equals -log2 of
    the purity sum p^2 of the charge-resolved operator Schmidt spectrum,
    computed from the brute-force rho by traces of the charge-sector blocks
    (sum sigma^4 = sum_q ||X_q^dag X_q||_F^2, no eigenvalues); alpha -> 1
    tends to the EE."""
    import itertools
    M, d = 3, 4
    rhos = _bounded_rhos(M, d, 3)
    U = inputs.haar_unitary(M, 4)
    gates, _ = clements.decompose(U)
    m = mpo.DenseMPO.product(rhos, 10 ** 6)
    rho = brute.product_rho(rhos)
    for (k, th, ph) in gates:
        m.apply_gate(k, th, ph, 10 ** 6)
        rho = brute.apply_gate(rho, k, th, ph)
    perm = []
    for j in range(M):
        perm += [j, M + j]
    v = np.transpose(rho, perm)
    R2 = m.renyi(2.0)
    for b in range(1, M):
        left = v.reshape(d ** (2 * b), d ** (2 * (M - b)))
        cols = {}
        for idx, cfg in enumerate(itertools.product(range(d), repeat=2 * (M - b))):
            cols.setdefault((sum(cfg[0::2]), sum(cfg[1::2])), []).append(idx)
        s4 = sum(np.linalg.norm(left[:, c].conj().T @ left[:, c]) ** 2 for c in cols.values())
        s2 = np.linalg.norm(left) ** 2
        assert abs(R2[b - 1] + np.log2(s4 / s2 ** 2)) < 1e-10
    assert np.abs(m.renyi(1.0 + 1e-8) - m.entropies()).max() < 1e-6


def _project_total(rho, K):
    """Brute force: keep only ket and bra configurations with at most K photons."""
    M = rho.ndim // 2
    d = rho.shape[0]
    n = np.indices((d,) * M).sum(axis=0)
    ok = n <= K
    mask = ok.reshape(ok.shape + (1,) * M) & ok.reshape((1,) * M + ok.shape)
    return np.where(mask, rho, 0.0)


@pytest.mark.parametrize("M,d,K,r,eta,seed", [(3, 4, 3, [0.8, 0.5, 0.0], 0.6, 31),
                                              (4, 3, 2, [0.9, 0.7, 0.4, 0.0], 0.5, 32),
                                              (3, 5, 4, [1.0, 0.9, 0.3], 0.45, 33)])
def test_total_photon_cap(M, d, K, r, eta, seed):
    """Global photon cap (App. A reading: the cutoff bounds the total photon
    number).  The closed-form initial state equals the dense sweeps and the
    brute-force projection onto at most K photons in ket and bra; since the
    interferometer conserves photon number, the projection commutes with it:
    untruncated runs equal U (P rho P) U^dag entrywise and the trace is
    exactly conserved (no photon leaves the cutoff)."""
    rhos = [states.lossy_squeezed_rho(x, eta, d) for x in r]
    m = mpo.DenseMPO.product(rhos, 10 ** 6, total_cap=K)
    s = mpo.DenseMPO.product_by_sweeps(rhos, 10 ** 6, total_cap=K)
    for b in range(M + 1):
        assert np.array_equal(m.charge[b], s.charge[b])
        assert np.allclose(m.lam[b], s.lam[b], rtol=1e-10, atol=1e-14)
        assert np.all(m.charge[b] <= K)
    rho = _project_total(brute.product_rho(rhos), K)
    assert np.abs(m.to_dense() - rho).max() < 1e-13
    _, tr0, _ = m.marginals()
    assert abs(tr0 - np.trace(rho.reshape(d ** M, d ** M)).real) < 1e-13
    U = inputs.haar_unitary(M, seed)
    gates, _ = clements.decompose(U)
    for (k, th, ph) in gates:
        m.apply_gate(k, th, ph, 10 ** 6)
        rho = brute.apply_gate(rho, k, th, ph)
        _, tr, _ = m.marginals()
        assert abs(tr - tr0) < 1e-13
    assert np.abs(m.to_dense() - rho).max() < 1e-12
    # the cap is what removes the leak: the per-mode cutoff alone loses trace
    free = mpo.DenseMPO.product(rhos, 10 ** 6)
    _, tf0, _ = free.marginals()
    for (k, th, ph) in gates:
        free.apply_gate(k, th, ph, 10 ** 6)
    assert free.marginals()[1] < tf0 - 1e-6
