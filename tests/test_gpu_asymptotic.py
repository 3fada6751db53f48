"""GPU parity of the Renyi readout (Sec. III.B) and of the App. C asymptotic
single-mode estimator, through the C ABI, against the FP64 oracle."""
import math

import numpy as np
import pytest

from oracle import asymptotic as oa, clements as oclem, mpo as omp, states
from paper_2301_12814_amd import gbsmpo, inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("r,mu,n_max,alpha,theta", [
    (0.88, 0.5, 12, 1.0, math.pi / 4), (0.88, 0.5, 12, 2.0, math.pi / 4),
    (0.88, 0.5, 12, 0.5, math.pi / 4), (1.1, 0.3, 20, 1.0, math.pi / 4),
    (0.5, 1.0, 16, 1.0, math.pi / 4), (0.9, 0.45, 14, 1.0, 0.6), (0.7, 0.05, 10, 3.0, math.pi / 4),
    (1.2, 0.8, 31, 1.0, math.pi / 4)])
def test_gpu_asymptotic_estimate_matches_oracle(r, mu, n_max, alpha, theta):
    n_inputs = 7
    S, spec = gbsmpo.asymptotic_ee(r, mu, n_max, n_inputs, alpha, theta)
    oS = oa.estimate(r, mu, n_max, n_inputs, alpha, theta)
    op = np.sort(oa.operator_spectrum(r, mu, n_max, theta))[::-1]
    p = np.sort(spec)[::-1]
    print("asymptotic", r, mu, n_max, alpha, "gpu", S, "oracle", oS, flush=True)
    assert abs(spec.sum() - 1.0) < 1e-13
    assert np.abs(p - op).max() < 1e-13
    tol = 1e-10 if alpha >= 1.0 else 1e-8
    assert abs(S - oS) < tol * n_inputs


def test_gpu_asymptotic_lossless_closed_form():
    """mu = 1: twice the entropy of the geometric spectrum with
    nbar = (cosh r - 1) / 2 (split squeezed vacuum, Gaussian closed form)."""
    r = 0.3
    nbar = (math.cosh(r) - 1) / 2
    want = 2 * ((nbar + 1) * math.log2(nbar + 1) - nbar * math.log2(nbar))
    S, _ = gbsmpo.asymptotic_ee(r, 1.0, 30, 1)
    assert abs(S - want) < 1e-12


def test_gpu_asymptotic_rejects_bad_arguments():
    for args in [(0.5, 0.0, 10, 1), (0.5, 1.5, 10, 1), (0.5, 0.5, 0, 1), (0.5, 0.5, 32, 1),
                 (-0.1, 0.5, 10, 1)]:
        with pytest.raises(gbsmpo.GbsMpoError) as ei:
            gbsmpo.asymptotic_ee(*args)
        assert ei.value.code == gbsmpo.MPO_EINVAL


def test_gpu_renyi_readout_matches_oracle():
    """Small workload (8 modes, d=4, chi=32), after three layers: Renyi-alpha
    of every internal bond for several alpha; alpha = 1 equals the EE."""
    w = inputs.workload("small")
    U = inputs.haar_unitary(w.M, w.seed)
    layers, _ = gbsmpo.clements(U)
    olayers = oclem.layers(w.M, oclem.decompose(U)[0])
    o = omp.DenseMPO.product([states.lossy_squeezed_rho(x, w.eta, w.d) for x in w.r], w.chi)
    with gbsmpo.MPO(w.M, w.r, w.eta, w.d, w.chi) as g:
        for li in range(3):
            g.apply_layer(*layers[li])
            for (k, th, ph) in olayers[li]:
                o.apply_gate(k, th, ph, w.chi)
        for alpha in (0.0, 0.5, 2.0, 3.0):
            assert np.abs(g.renyi(alpha) - o.renyi(alpha)).max() < 1e-10, alpha
        S, _ = g.entropy()
        assert np.abs(g.renyi(1.0) - S).max() < 1e-13
