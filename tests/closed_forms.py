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
