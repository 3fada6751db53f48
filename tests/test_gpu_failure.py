"""Failure isolation in a batch (host-forced, every kernel exits normally):
one simulation whose Jacobi sweep limit is lowered to 1 latches MPO_ENUMERIC
and is retired with that error, while the other simulations of the same
batched launches finish with results bitwise equal to their runs alone; an
admission refused mid-batch for lack of budget leaves the running
simulations unchanged."""
import numpy as np
import pytest

from paper_2301_12814_amd import gbsmpo, inputs

pytestmark = pytest.mark.gpu

SPECS = [(6, 0.6, 0.5, 4, 16, 50), (8, 0.5, 0.5, 4, 32, 51), (7, 0.4, 0.6, 6, 20, 54)]


def _alone(M, r, eta, d, chi, seed):
    layers, _ = gbsmpo.clements(inputs.haar_unitary(M, seed))
    with gbsmpo.MPO(M, r, eta, d, chi) as g:
        for L in layers:
            g.apply_layer(*L)
        _, smax = g.entropy()
        P, tr = g.marginals()
    return smax, tr, P


def _run(eng, ids):
    steps = 0
    while any(eng.result(s) is None for s in ids if not _failed(eng, s)):
        eng.step()
        steps += 1
        assert steps < 100


def _failed(eng, sid):
    try:
        eng.result(sid)
        return False
    except gbsmpo.GbsMpoError:
        return True


def test_gpu_one_failing_simulation_leaves_the_others_unchanged():
    alone = [_alone(M, r, eta, d, chi, s) for (M, r, eta, d, chi, s) in SPECS]
    with gbsmpo.Engine() as eng:
        ids = [eng.add(M, r, eta, d, chi, inputs.haar_unitary(M, s))
               for (M, r, eta, d, chi, s) in SPECS]
        eng.set_sweep_limit(ids[1], 1)
        _run(eng, ids)
        with pytest.raises(gbsmpo.GbsMpoError) as ei:
            eng.result(ids[1])
        assert ei.value.code == gbsmpo.MPO_ENUMERIC
        assert "converge" in str(ei.value)
        for k in (0, 2):
            res = eng.result(ids[k])
            smax, tr, P = alone[k]
            assert res["S_max"] == smax and res["trace"] == tr, k
            assert np.array_equal(res["P"], P), k


def test_gpu_admission_refused_mid_batch():
    (M, r, eta, d, chi, s) = SPECS[0]
    smax, tr, P = _alone(M, r, eta, d, chi, s)
    budget = gbsmpo.projected_bytes(M, d, chi) + gbsmpo.projected_bytes(8, 4, 32) // 2
    with gbsmpo.Engine(budget_bytes=budget) as eng:
        sid = eng.add(M, r, eta, d, chi, inputs.haar_unitary(M, s))
        eng.step()
        eng.step()
        with pytest.raises(gbsmpo.GbsMpoError) as ei:
            eng.add(8, 0.5, 0.5, 4, 32, inputs.haar_unitary(8, 1))
        assert ei.value.code == gbsmpo.MPO_ENOMEM
        _run(eng, [sid])
        res = eng.result(sid)
        assert res["S_max"] == smax and res["trace"] == tr
        assert np.array_equal(res["P"], P)
