"""Closed forms fixed by the mathematics, used to pin the oracle.

None of these is oracle code; each is an independent formula:

* Photon-number generating function of a single-mode zero-mean Gaussian state
  with <a^dag a> = N and |<a a>| = A:
  G(z) = sum_n P(n) z^n = ((1 + (1 - z) N)^2 - (1 - z)^2 A^2)^(-1/2).
  Squeezed vacuum has N = sinh^2 r, A = sinh r cosh r; loss with
  transmission eta thins both by eta (binomial thinning z -> 1 - eta + eta z).
* Purity of that state: Tr rho^2 = ((1 + 2N)^2 - 4 A^2)^(-1/2).
"""
import math

import numpy as np


def series_inv_sqrt(g0: float, g1: float, g2: float, n_terms: int) -> np.ndarray:
    """Taylor coefficients of (g0 + g1 z + g2 z^2)^(-1/2).

    From f = g^(-1/2):  g f' = -(1/2) g' f, coefficient of z^n gives
    g0 (n+1) f_{n+1} = -(n + 1/2) g1 f_n - n g2 f_{n-1}.
    """
    f = np.zeros(n_terms)
    f[0] = g0 ** -0.5
    for n in range(n_terms - 1):
        prev = f[n - 1] if n >= 1 else 0.0
        f[n + 1] = -((n + 0.5) * g1 * f[n] + n * g2 * prev) / (g0 * (n + 1))
    return f


def gaussian_photon_distribution(N: float, A: float, n_terms: int) -> np.ndarray:
    """P(n) for a zero-mean single-mode Gaussian state (<a^dag a>=N, |<aa>|=A)."""
    # (1 + (1-z) N)^2 - (1-z)^2 A^2 with u = 1 - z:
    # (1 + N)^2 - 2 (1 + N) N z + N^2 z^2 - A^2 (1 - 2 z + z^2)
    g0 = (1 + N) ** 2 - A ** 2
    g1 = -2 * (1 + N) * N + 2 * A ** 2
    g2 = N ** 2 - A ** 2
    return series_inv_sqrt(g0, g1, g2, n_terms)


def lossy_squeezed_moments(r: float, eta: float):
    s, c = math.sinh(r), math.cosh(r)
    return eta * s * s, eta * s * c


def lossy_squeezed_distribution(r: float, eta: float, n_terms: int) -> np.ndarray:
    N, A = lossy_squeezed_moments(r, eta)
    return gaussian_photon_distribution(N, A, n_terms)


def gaussian_purity(N: float, A: float) -> float:
    return ((1 + 2 * N) ** 2 - 4 * A * A) ** -0.5


def output_mode_moments(U: np.ndarray, r, eta: float):
    """<b_i^dag b_i> and |<b_i b_i>| after loss then the interferometer U
    (a_j^dag -> sum_i U[i, j] a_i^dag)."""
    r = np.asarray(r, dtype=float)
    n_in = eta * np.sinh(r) ** 2
    m_in = eta * np.sinh(r) * np.cosh(r)
    N = (np.abs(U) ** 2) @ n_in
    A = np.abs((U ** 2) @ m_in)
    return N, A


def gaussian_rho(N: float, A: complex, d: int, K: int = 96) -> np.ndarray:
    """Fock matrix [0, d)^2 of the zero-mean single-mode Gaussian state with
    <a^dag a> = N and <a a> = A (complex), built as a squeezed thermal state
    S(z) rho_th S(z)^dag in a K-level Fock space by matrix exponentials.

    With S(z) = exp((conj(z) a^2 - z a^dag^2) / 2), z = t e^{i th}:
    S^dag a S = a cosh t - a^dag e^{i th} sinh t, so for a thermal state of
    mean n_th, with nu = n_th + 1/2:
        <a^dag a> = nu cosh 2t - 1/2,   <a a> = -nu e^{i th} sinh 2t,
    hence nu = sqrt((N + 1/2)^2 - |A|^2), cosh 2t = (N + 1/2) / nu and
    e^{i th} = -A / |A|.  The levels used (n < d) are far from the K-level
    edge, so the truncation of the exponential does not reach them.
    """
    from scipy.linalg import expm

    nu = math.sqrt((N + 0.5) ** 2 - abs(A) ** 2)
    nth = nu - 0.5
    t = 0.5 * math.acosh(max((N + 0.5) / nu, 1.0))
    eth = -A / abs(A) if abs(A) > 0 else 1.0
    z = t * eth
    a = np.diag(np.sqrt(np.arange(1, K)), 1).astype(complex)
    ad = a.conj().T
    S = expm(0.5 * (np.conj(z) * (a @ a) - z * (ad @ ad)))
    x = nth / (nth + 1.0)
    th = np.diag((1.0 - x) * x ** np.arange(K)).astype(complex)
    rho = S @ th @ S.conj().T
    return rho[:d, :d]


def output_mode_coherences(U: np.ndarray, r, eta: float):
    """<b_i^dag b_i> and the complex <b_i b_i> after loss then the
    interferometer U (a_j^dag -> sum_i U[i, j] a_i^dag): with independent
    inputs, U^dag b_i U = sum_j U[i, j] a_j gives <b_i b_i> = sum_j U[i, j]^2
    <a_j a_j>, and <a a> = eta sinh r cosh r for the squeezed vacuum with
    positive amplitudes thinned by the loss."""
    r = np.asarray(r, dtype=float)
    n_in = eta * np.sinh(r) ** 2
    m_in = eta * np.sinh(r) * np.cosh(r)
    return (np.abs(U) ** 2) @ n_in, (U ** 2) @ m_in
