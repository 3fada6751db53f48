"""Pins of the oracle's App. C asymptotic estimator and of the Renyi entropies.

* Lossless input (mu = 1): the split squeezed vacuum is a pure two-mode
  Gaussian state; the up mode's reduced state has covariance
  (1 + e^{-2r}, 1 + e^{2r}) / 2 (vacuum = 1), symplectic eigenvalue cosh r, so
  its spectrum is geometric with mean nbar = (cosh r - 1) / 2.  The vectorised
  operator |psi>|psi*> has the product of two such spectra: every Renyi entropy
  is twice the Gaussian one (closed form, independent of the Fock algebra).
* A beam splitter from the two-mode Fock matrix (the oracle's own fock module,
  built by a different route: the binomial expansion of the creation
  operators) acting on the lossy input and a vacuum gives the same spectrum as
  the estimator's transform (App. B Eq. transform) at every loss.
* Limits: no split (theta = 0) and vanishing transmission give zero entropy;
  at small transmission the entropy scales as mu^2 log(1/mu) (App. B).
* Renyi entropies: alpha -> 1 tends to the von Neumann value, alpha = 0 counts
  the support, alpha = 2 equals -log2 of the purity sum p^2 computed from the
  trace of the squared reduced operator (no eigenvalues involved).
"""
import math

import numpy as np
import pytest

from oracle import asymptotic as oa, fock


def gaussian_renyi(nbar, alpha):
    x = nbar / (nbar + 1.0)
    if alpha == 1.0:
        return (nbar + 1) * math.log2(nbar + 1) - (nbar * math.log2(nbar) if nbar > 0 else 0.0)
    return (alpha * math.log2(1 - x) - math.log2(1 - x ** alpha)) / (1 - alpha)


@pytest.mark.parametrize("r,alpha,tol", [(0.3, 1.0, 1e-13), (0.5, 1.0, 1e-9), (0.3, 2.0, 1e-13),
                                         (0.3, 3.0, 1e-13), (0.2, 0.5, 1e-9)])
def test_lossless_split_matches_gaussian_closed_form(r, alpha, tol):
    nbar = (math.cosh(r) - 1) / 2
    got = oa.estimate(r, 1.0, 30, 1, alpha)
    assert abs(got - 2 * gaussian_renyi(nbar, alpha)) < tol


@pytest.mark.parametrize("r,mu", [(0.88, 0.5), (1.1, 0.3), (0.6, 0.9)])
def test_transform_equals_a_fock_beam_splitter_on_input_and_vacuum(r, mu):
    n_max = 10
    L = n_max + 1
    rho = oa.lossy_input(r, mu, n_max)
    T = fock.bs_matrix(math.pi / 4, 0.0)                    # a0^dag -> (a_u^dag + a_d^dag)/sqrt2
    Uf = fock.fock_bs(T, L)                                 # [I, J, i, j], cutoff L per mode
    vac = np.zeros((L, L))
    vac[0, 0] = 1.0
    rho2 = np.einsum('IJij,ik,jl,KLkl->IJKL', Uf, rho, vac, Uf.conj())
    X = np.transpose(rho2, (0, 2, 1, 3)).reshape(L * L, L * L)
    sv2 = np.linalg.svd(X, compute_uv=False) ** 2
    p_ref = np.sort(sv2 / sv2.sum())[::-1]
    p = np.sort(oa.operator_spectrum(r, mu, n_max))[::-1]
    assert np.abs(p - p_ref).max() < 1e-13
    assert abs(oa.renyi(p, 1.0) - oa.renyi(p_ref, 1.0)) < 1e-12


def test_limits_and_small_loss_scaling():
    assert oa.estimate(0.9, 0.7, 12, 5, theta=0.0) == pytest.approx(0.0, abs=1e-14)
    assert oa.estimate(0.9, 1e-6, 12, 1) < 1e-10
    ratios = [oa.estimate(0.88, mu, 16, 1) / (mu ** 2 * math.log2(1 / mu)) for mu in (3e-3, 1e-3)]
    assert abs(ratios[0] / ratios[1] - 1) < 0.01
    # additivity over inputs
    assert oa.estimate(0.7, 0.4, 12, 7) == pytest.approx(7 * oa.estimate(0.7, 0.4, 12, 1), rel=1e-14)


def test_renyi_special_values():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((9, 7))
    sv2 = np.linalg.svd(X, compute_uv=False) ** 2
    p = sv2 / sv2.sum()
    assert oa.renyi(p, 1.0 + 1e-7) == pytest.approx(oa.renyi(p, 1.0), abs=1e-6)
    assert oa.renyi(p, 0.0) == pytest.approx(math.log2(7), abs=1e-14)
    red = X.T @ X
    purity = np.trace(red @ red) / np.trace(red) ** 2
    assert oa.renyi(p, 2.0) == pytest.approx(-math.log2(purity), abs=1e-13)
