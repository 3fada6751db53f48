"""GPU parity at the sizes of the workloads themselves.

A dense oracle cannot hold the two-site tensor at chi = 256 or 1024 (a dense
Theta is (chi d^2)^2 complex numbers), so full-size gates are checked gate by
gate: the library's own state before a layer is read back, the oracle forms
EVERY charge sector Theta(q) of a gate from it (App. D, Eq. theta, in the
blocked form), takes all their singular values, applies the truncation rule
(rank cut, mirror-pair units, top chi) and the result must equal the bond the
library wrote: kept charges bit-exact, values within 1e-10 relative (plus
1e-12 of the bond maximum).  When the chi-th and the first dropped unit are
closer than 1e-8 relative (a degenerate cut, where rounding may pick either),
only the values above the cut are compared and the case is printed.

The batch-law instances with cutoff d = 10 are run layer by layer against the
dense oracle at a reduced chi.
"""
import sys

import numpy as np
import pytest

from oracle import clements as oclem, mpo as omp, states
from paper_2301_12814_amd import gbsmpo, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_gate_bond(before, th, ph, d, chi):
    """(charges, values) of the new centre bond that the oracle selects from
    every sector of the gate, plus (cut value, best dropped value)."""
    (lL, cL), (lC, cC), (lR, cR), Gj, Gj1 = before
    qs = {tuple(int(x) for x in (a - np.array([m0, m1])))
          for a in np.unique(cL, axis=0) for m0 in range(d) for m1 in range(d)}
    vals, chs = [], []
    nsec = 0
    for q in sorted(qs):
        rows, cols, Th = omp.sector_theta(Gj, Gj1, lL, lC, lR, cL, cC, cR, th, ph, d,
                                          np.array(q))
        if Th.size == 0:
            continue
        nsec += 1
        s = np.linalg.svd(Th, compute_uv=False)
        vals.extend(s.tolist())
        chs.extend([q] * len(s))
    vals = np.array(vals)
    chs = np.array(chs, dtype=int).reshape(-1, 2)
    keep = omp.select(chs, vals, chi)
    dropped = np.setdiff1d(np.arange(len(vals)), keep)
    dropped = dropped[vals[dropped] >= omp.RANK_CUT * vals.max()]
    best_drop = float(vals[dropped].max()) if len(dropped) else 0.0
    return chs[keep], vals[keep], float(vals[keep].min()), best_drop, nsec


def check_gate(before, th, ph, d, chi, lam, ch, ctx):
    och, oval, vcut, vdrop, nsec = oracle_gate_bond(before, th, ph, d, chi)
    degenerate = vdrop > 0 and (vcut - vdrop) <= 1e-8 * vcut
    say(ctx, "sectors", nsec, "kept", len(oval), "cut", vcut, "best dropped", vdrop,
        "degenerate cut" if degenerate else "")
    if not degenerate:
        assert np.array_equal(ch, och), ctx
        sel_l, sel_o = np.ones(len(lam), bool), np.ones(len(oval), bool)
    else:
        thr = vdrop * (1 + 1e-8)
        sel_l, sel_o = lam > thr, oval > thr
        assert np.array_equal(ch[sel_l], och[sel_o]), ctx
    err = np.abs(lam[sel_l] - oval[sel_o])
    tol = 1e-10 * oval[sel_o] + 1e-12 * oval.max()
    assert np.all(err <= tol), (ctx, float((err / tol).max()))


def run_and_check(w, layer, gate_ids):
    U = inputs.haar_unitary(w.M, w.seed)
    layers, _ = gbsmpo.clements(U)
    with gbsmpo.MPO(w.M, w.r, w.eta, w.d, w.chi) as g:
        for li in range(layer):
            g.apply_layer(*layers[li])
        S, T, P = layers[layer]
        sel = [(int(S[k]), float(T[k]), float(P[k])) for k in gate_ids(len(S))]
        before = {}
        for (j, th, ph) in sel:
            before[j] = (g.bond(j), g.bond(j + 1), g.bond(j + 2), g.site(j), g.site(j + 1))
        g.apply_layer(S, T, P)
        after = {j: g.bond(j + 1) for (j, _, _) in sel}
    for (j, th, ph) in sel:
        lam, ch = after[j]
        check_gate(before[j], th, ph, w.d, w.chi, lam, ch, f"{w.name} layer {layer} gate at {j}")


@pytest.mark.timeout(900)
def test_gpu_medium_full_chi_every_sector():
    """Medium workload (M=32, r=0.8, d=8, chi=256) at full chi: after six
    layers, two gates of the seventh (the middle one and the last one)."""
    run_and_check(inputs.workload("medium"), 6, lambda n: [n // 2, n - 1])


@pytest.mark.timeout(900)
def test_gpu_large_full_chi_every_sector():
    """Large workload (M=64, r=0.9, eta=0.3, d=8, chi=1024), the configuration
    the benchmark times: after seven layers, the middle gate of the eighth,
    every sector and the kept set."""
    run_and_check(inputs.workload("large"), 7, lambda n: [n // 2])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("idx,chi", [(148, 10), (68, 12)])
def test_gpu_batch_law_cutoff_10_matches_oracle(idx, chi):
    """Batch-law instances with Fock cutoff d = 10 (M = 16 and 18), chi
    reduced so that the dense oracle stays fast: the first four layers, every
    bond after every layer, and marginals, against the oracle."""
    w = inputs.batch_workloads(idx + 1)[idx]
    U = inputs.haar_unitary(w.M, w.seed)
    layers, _ = gbsmpo.clements(U)
    olayers = oclem.layers(w.M, oclem.decompose(U)[0])
    o = omp.DenseMPO.product([states.lossy_squeezed_rho(x, w.eta, w.d) for x in w.r], chi)
    with gbsmpo.MPO(w.M, w.r, w.eta, w.d, chi) as g:
        for li in range(4):
            g.apply_layer(*layers[li])
            for (k, th, ph) in olayers[li]:
                o.apply_gate(k, th, ph, chi)
            for b in range(w.M + 1):
                lam, ch = g.bond(b)
                assert np.array_equal(ch, o.charge[b]), (idx, li, b)
                err = np.abs(lam - o.lam[b])
                assert np.all(err <= 1e-10 * o.lam[b] + 1e-12 * o.lam[b].max()), (idx, li, b)
            S, _ = g.entropy()
            assert np.abs(S - o.entropies()).max() < 1e-10, (idx, li)
            say("batch instance", idx, "layer", li, "ok")
        P, tr = g.marginals()
    oP, otr, _ = o.marginals()
    assert abs(tr - otr) < 1e-10 * abs(otr)
    assert np.abs(P - oP).max() < 1e-10
