"""The library's count of algorithmic contraction flops (the roofline
numerator of the contraction) against an independent count from the bond
charges read back through the C ABI."""
import numpy as np
import pytest

from paper_2301_12814_amd import gbsmpo, inputs

pytestmark = pytest.mark.gpu


def _gate_flops(cL, cC, cR, d):
    def valid(x):
        return np.all((x >= 0) & (x < d), axis=-1)
    LC = valid(cL[:, None, :] - cC[None, :, :])            # (a, alpha)
    CR = valid(cC[:, None, :] - cR[None, :, :])            # (alpha, b)
    sums = 8.0 * float((LC.sum(axis=0) * CR.sum(axis=1)).sum())
    n = cL[:, None, :] - cR[None, :, :]                     # (a, b, 2)
    ok = np.all((n >= 0) & (n <= 2 * d - 2), axis=-1)
    m = np.minimum(n, 2 * d - 2 - n) + 1
    mk, mb = m[..., 0], m[..., 1]
    weights = 8.0 * float((mk * mb * (mk + mb))[ok].sum())
    return sums + weights


@pytest.mark.parametrize("name,layers", [("small", 3), ("medium", 2)])
def test_gpu_contraction_flop_count(name, layers):
    w = inputs.workload(name)
    L, _ = gbsmpo.clements(inputs.haar_unitary(w.M, w.seed))
    with gbsmpo.MPO(w.M, w.r, w.eta, w.d, w.chi) as g:
        for li in range(layers):
            g.apply_layer(*L[li])
        S, T, P = L[layers]
        want = 0.0
        for k in S:
            k = int(k)
            want += _gate_flops(g.bond(k)[1], g.bond(k + 1)[1], g.bond(k + 2)[1], w.d)
        g.set_profiling(True)
        g.apply_layer(S, T, P)
        got = g.contraction_flops()
    assert got == pytest.approx(want, rel=1e-12)
