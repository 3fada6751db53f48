"""Asymptotic single-mode estimate of the operator entanglement entropy and
the Renyi entropies (oracle, FP64, dense).

Test infrastructure only (see ``oracle/__init__``).

App. C: for system sizes where direct MPO runs are impractical, the EE is
estimated from one input mode.  The lossy squeezed input (App. C input
wavefunction, App. B Kraus operators, both truncated to photon numbers
0..n_max) is sent through the basis transform of App. B (Eq. transform):

    |n> -> sum_k sqrt(binom(n, k)) cos^k(t) sin^(n-k)(t) |k>_u |n-k>_d,

which splits the mode into the parts of the interferometer's output on the
two sides of the cut ("up" and "down" modes); App. C takes cos t = sin t =
1/sqrt(2) for the middle cut of a large random interferometer.  The output
operator rho_out[k_u, k_d; k'_u, k'_d] is vectorised, |rho>> grouped as
(K_u = (k_u, k'_u)) x (K_d = (k_d, k'_d)), the reduced operator of the outer
product over the up side is formed, its eigenvalues are normalised, and the
entropy is taken; the system estimate is that entropy times the number of
squeezed inputs (the output is a product over inputs, App. B).

Renyi entropies of the same normalised spectrum (Sec. III.B, App. B):
S_alpha = log2(sum p^alpha) / (1 - alpha); alpha = 1 is the von Neumann value
-sum p log2 p.
"""
from __future__ import annotations

import math

import numpy as np

from . import states


def renyi(p: np.ndarray, alpha: float) -> float:
    """Renyi-alpha entropy in bits of a distribution p (normalised here);
    alpha = 1 gives -sum p log2 p, alpha = 0 gives log2 of the support size."""
    p = np.asarray(p, dtype=float)
    p = p / p.sum()
    p = p[p > 0]
    if alpha == 1.0:
        return float(-(p * np.log2(p)).sum())
    return float(math.log2((p ** alpha).sum()) / (1.0 - alpha))


def lossy_input(r: float, mu: float, n_max: int) -> np.ndarray:
    """rho_lossy on photon numbers 0..n_max: the squeezed vacuum and the loss
    Kraus operators both truncated to that space (App. C)."""
    psi = states.squeezed_vacuum(r, n_max + 1)
    return states.apply_loss(np.outer(psi, psi), mu)


def split_amplitude(n: int, k: int, theta: float) -> float:
    """<k_u = k, k_d = n - k | U | n> of the basis transform (App. B, Eq. kun)."""
    return math.sqrt(math.comb(n, k)) * math.cos(theta) ** k * math.sin(theta) ** (n - k)


def output_operator(r: float, mu: float, n_max: int, theta: float = math.pi / 4) -> np.ndarray:
    """rho_out[k_u, k_d, k'_u, k'_d] = sum_{m,n} <k_u k_d|U|m> rho_lossy[m, n]
    <n|U^dag|k'_u k'_d> (App. B, the output operator in the bipartition basis)."""
    rho = lossy_input(r, mu, n_max)
    L = n_max + 1
    T = np.zeros((L, L, L))                 # T[k_u, k_d, m]
    for m in range(L):
        for k in range(m + 1):
            T[k, m - k, m] = split_amplitude(m, k, theta)
    return np.einsum('abm,mn,cdn->abcd', T, rho, T)


def operator_spectrum(r: float, mu: float, n_max: int, theta: float = math.pi / 4):
    """Normalised eigenvalues of tr_u(|rho_out>><<rho_out|) (App. C).  With the
    vectorised operator written as the matrix X[K_u, K_d], that reduced
    operator is X^T conj(X), whose eigenvalues are the squared singular
    values of X; they are taken from the SVD of X, which resolves small
    eigenvalues far below the rounding of the product X^T X."""
    out = output_operator(r, mu, n_max, theta)
    L = n_max + 1
    X = np.transpose(out, (0, 2, 1, 3)).reshape(L * L, L * L)   # [(k_u, k'_u), (k_d, k'_d)]
    ev = np.linalg.svd(X, compute_uv=False) ** 2
    return ev / ev.sum()


def estimate(r: float, mu: float, n_max: int, n_inputs: int, alpha: float = 1.0,
             theta: float = math.pi / 4) -> float:
    """App. C estimate of the system's operator EE (alpha = 1) or Renyi-alpha
    entropy: the single-mode value times the number of squeezed inputs."""
    return n_inputs * renyi(operator_spectrum(r, mu, n_max, theta), alpha)
