"""Per-mode input states of lossy Gaussian boson sampling (oracle, FP64).

Test infrastructure only (see ``oracle/__init__``).

* Single-mode squeezed vacuum, App. C (input wavefunction): amplitude of
  |2n> is tanh(r)^n * sqrt((2n)!) / (2^n n!) / sqrt(cosh r), because
  a^dag^{2n}|0> = sqrt((2n)!) |2n>.  The sign is +tanh(r)^n exactly as printed.
* Pure loss with transmission eta, App. B (Kraus operators): K^(l) maps
  |n_in> to |n_out = n_in - l> with amplitude
  sqrt(binom(n_in, n_out) eta^n_out (1-eta)^l), and rho -> sum_l K rho K^dag.
* Uniform loss commutes with the interferometer (Sec. II; App. B), so the
  whole loss is applied here, to the input state, before any beam splitter.

The state is built in a large internal Fock space (tail probability below
1e-20), the loss is applied there, and only then is the result cropped to the
per-mode cutoff d.  Nothing is renormalised.
"""
from __future__ import annotations

import math

import numpy as np


def internal_cutoff(r: float, d: int, tail: float = 1e-20) -> int:
    """Smallest even-extended Fock dimension whose squeezed tail is < ``tail``."""
    if r == 0.0:
        return max(d, 2)
    t2 = math.tanh(r) ** 2
    n = 0
    while True:
        # |psi_{2n}|^2 upper bound ~ t2^n / sqrt(pi n) / cosh r
        logp = n * math.log(t2) + (math.lgamma(2 * n + 1) - 2 * n * math.log(2.0)
                                   - 2 * math.lgamma(n + 1)) - math.log(math.cosh(r))
        if 2 * n + 1 >= d and logp < math.log(tail):
            return 2 * n + 2
        n += 1


def squeezed_vacuum(r: float, n_int: int) -> np.ndarray:
    """Fock amplitudes psi[0..n_int-1] of the squeezed vacuum (App. C)."""
    psi = np.zeros(n_int)
    t = math.tanh(r)
    for n in range(0, (n_int + 1) // 2):
        k = 2 * n
        if k >= n_int:
            break
        if t == 0.0:
            amp_log = 0.0 if n == 0 else -math.inf
        else:
            amp_log = (n * math.log(abs(t)) + 0.5 * math.lgamma(k + 1)
                       - n * math.log(2.0) - math.lgamma(n + 1))
        sign = 1.0 if (t >= 0 or n % 2 == 0) else -1.0
        psi[k] = sign * math.exp(amp_log) / math.sqrt(math.cosh(r))
    return psi


def loss_kraus(eta: float, n_int: int, l: int) -> np.ndarray:
    """Kraus operator K^(l) as an (n_int x n_int) matrix [n_out, n_in] (App. B)."""
    K = np.zeros((n_int, n_int))
    for n_out in range(0, n_int - l):
        n_in = n_out + l
        if eta == 1.0:
            val = 1.0 if l == 0 else 0.0
        else:
            logv = (math.lgamma(n_in + 1) - math.lgamma(n_out + 1) - math.lgamma(l + 1)
                    + (n_out * math.log(eta) if n_out > 0 else 0.0)
                    + (l * math.log(1.0 - eta) if l > 0 else 0.0))
            val = math.exp(0.5 * logv)
        K[n_out, n_in] = val
    return K


def apply_loss(rho_in: np.ndarray, eta: float) -> np.ndarray:
    """rho -> sum_l K^(l) rho K^(l)^dag over every loss count l (App. B).

    K^(l) has a single shifted diagonal k_l[m] = K^(l)[m, m+l], so each term is
    (K rho K^dag)[m, n] = k_l[m] rho[m+l, n+l] k_l[n]; this is the index form
    the appendix writes in its second line of the lossy-state equation.
    """
    n_int = rho_in.shape[0]
    out = np.zeros_like(rho_in)
    for l in range(n_int):
        K = loss_kraus(eta, n_int, l)
        k = np.array([K[m, m + l] for m in range(n_int - l)])
        out[: n_int - l, : n_int - l] += k[:, None] * rho_in[l:, l:] * k[None, :]
    return out


def lossy_squeezed_rho(r: float, eta: float, d: int, n_int: int | None = None) -> np.ndarray:
    """Per-mode density matrix rho_j (d x d, real symmetric), not renormalised.

    Squeezed vacuum (App. C) -> loss (App. B) in an internal Fock space of
    dimension ``n_int`` -> crop to [0, d)^2.  ``r = 0`` gives the vacuum.
    """
    if n_int is None:
        n_int = internal_cutoff(r, d)
    psi = squeezed_vacuum(r, n_int)
    rho_in = np.outer(psi, psi.conj())
    rho = apply_loss(rho_in, eta)
    return np.ascontiguousarray(rho[:d, :d])
