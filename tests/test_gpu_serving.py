"""Serving as the benchmark runs it: two engines on two HIP streams, each
stepped by its own host thread at the same time (their kernels overlap on the
device), simulations admitted while others run.  Every simulation's results
must be bitwise the same as its run alone on the single-simulation path."""
import threading

import numpy as np
import pytest

from paper_2301_12814_amd import gbsmpo, inputs

pytestmark = pytest.mark.gpu

LANES = [
    [(6, 0.6, 0.5, 4, 16, 60), (9, 0.8, 0.4, 5, 24, 61), (7, 0.5, 0.6, 6, 20, 62)],
    [(12, 0.9, 0.3, 6, 48, 63), (10, 0.7, 0.5, 4, 32, 64)],
]


def _alone(M, r, eta, d, chi, seed):
    layers, _ = gbsmpo.clements(inputs.haar_unitary(M, seed))
    with gbsmpo.MPO(M, r, eta, d, chi) as g:
        for L in layers:
            g.apply_layer(*L)
        _, smax = g.entropy()
        P, tr = g.marginals()
    return smax, tr, P


def test_gpu_two_concurrent_engines_match_alone_runs():
    want = {spec: _alone(*spec) for lane in LANES for spec in lane}
    got, errors = {}, []

    def lane(specs):
        try:
            with gbsmpo.Engine() as eng:
                ids, pending, step = {}, list(specs), 0
                while pending or any(eng.result(s) is None for s in ids.values()):
                    if pending and step % 3 == 0:          # arrivals between steps
                        spec = pending.pop(0)
                        M, r, eta, d, chi, seed = spec
                        ids[spec] = eng.add(M, r, eta, d, chi, inputs.haar_unitary(M, seed))
                    eng.step()
                    step += 1
                    assert step < 400
                for spec, sid in ids.items():
                    got[spec] = eng.result(sid)
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    th = [threading.Thread(target=lane, args=(specs,)) for specs in LANES]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for spec, (smax, tr, P) in want.items():
        res = got[spec]
        assert res["S_max"] == smax and res["trace"] == tr, spec
        assert np.array_equal(res["P"], P), spec
