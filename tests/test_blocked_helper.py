"""CPU check of the test helper that reads a charge-blocked MPO back into a
dense rho: on the oracle's dense Vidal MPO written in blocked form, it must
reproduce the brute-force density matrix."""
import numpy as np

from oracle import brute, clements as oclem, mpo as omp, states
from paper_2301_12814_amd import inputs
from tests.blocked import expand_site, library_rho


class _Blocked:
    """A DenseMPO seen through the library's accessors (bond / site)."""

    def __init__(self, o):
        self.o = o

    def bond(self, b):
        return self.o.lam[b], self.o.charge[b]

    def site(self, j):
        # the dense SVD's vectors are charge-definite up to rounding, which
        # V / lam magnifies where lam is small: compare with the largest entry
        o = self.o
        G = o.G[j]
        tol = 1e-10 * np.abs(G).max()
        cl, cr = o.charge[j], o.charge[j + 1]
        B = np.zeros((G.shape[0], G.shape[3]), dtype=complex)
        for a in range(G.shape[0]):
            for b in range(G.shape[3]):
                m, mp = cl[a] - cr[b]
                if 0 <= m < o.d and 0 <= mp < o.d:
                    B[a, b] = G[a, m, mp, b]
                    # every other local entry of a charge-definite tensor is 0
                    rest = np.abs(G[a, :, :, b]).sum() - abs(G[a, m, mp, b])
                    assert rest < tol
                else:
                    assert np.abs(G[a, :, :, b]).max() < tol
        return B


def test_library_rho_reads_blocked_form():
    M, d, eta = 3, 4, 0.6
    r = [0.7, 0.4, 0.9]
    U = inputs.haar_unitary(M, 11)
    og, oph = oclem.decompose(U)
    rhos = [states.lossy_squeezed_rho(x, eta, d) for x in r]
    o = omp.DenseMPO.product(rhos, 512)
    rho = brute.product_rho(rhos)
    for (k, th, ph) in og:
        o.apply_gate(k, th, ph, 512)
        rho = brute.apply_gate(rho, k, th, ph)
    o.apply_phases(oph)
    rho = brute.apply_phases(rho, oph)
    got, outside = library_rho(_Blocked(o), M, d)
    assert outside == 0.0
    assert np.abs(got - rho).max() < 1e-12
    # a conjugated phase screen is seen
    assert np.abs(got - brute.apply_phases(brute.apply_phases(rho, -oph), -oph)).max() > 1e-3


def test_expand_site_reports_entries_outside_the_pattern():
    cl = np.array([[1, 1], [0, 0]])
    cr = np.array([[0, 0]])
    G = np.array([[2.0 + 1j], [3.0]])
    T, out = expand_site(G, cl, cr, 2)
    assert out == 0.0 and T[0, 1, 1, 0] == 2.0 + 1j and T[1, 0, 0, 0] == 3.0
    _, out = expand_site(G, np.array([[2, 0], [0, 0]]), cr, 2)
    assert out == abs(2.0 + 1j)
