"""Host-side properties the measurements rely on (no GPU).

* The serving stream draws each request's arrival gap and kind from one
  seeded generator in a fixed order, so the requests do not depend on the
  rate: a stream at another rate holds the same simulations, only their
  arrival times scale.  The alone baseline of a serving run relies on it.
* bench.py reports the SVD stage's HBM traffic only from a PMC summary taken
  on the same kernels (source digest) and the same workload.
"""
import os

import numpy as np

import bench
from paper_2301_12814_amd import inputs


def test_serving_requests_do_not_depend_on_the_rate():
    a = inputs.serving_requests(120, 0.3)
    b = inputs.serving_requests(120, 0.6)
    assert len(a) == len(b) == 120
    for (ta, wa), (tb, wb) in zip(a, b):
        assert (wa.name, wa.M, wa.eta, wa.d, wa.chi, wa.seed) == (wb.name, wb.M, wb.eta, wb.d, wb.chi, wb.seed)
        assert np.array_equal(np.asarray(wa.r), np.asarray(wb.r))
        assert abs(tb - 0.5 * ta) <= 1e-12 * ta
    large = [w for _, w in a if w.chi >= 1024]
    assert large and all(w.M == 96 and w.d == 10 for w in large)


def test_stage_traffic_needs_the_same_kernels_and_workload(tmp_path, monkeypatch):
    digest = bench._sources_digest()
    good = tmp_path / "good.txt"
    good.write_text("# comment: 1\nhbm_bytes_per_stage: 1.5e+11\nsource_digest: %s\n" % digest)
    stale = tmp_path / "stale.txt"
    stale.write_text("hbm_bytes_per_stage: 1.5e+11\nsource_digest: 0000000000000000\n")
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(good))
    assert bench.stage_traffic("large", "fp64", 64) == 1.5e11
    assert bench.stage_traffic("large", "mixed", 64) is None
    assert bench.stage_traffic("table1", "fp64", 12) is None
    assert bench.stage_traffic("large", "fp64", 10) is None
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(stale))
    assert bench.stage_traffic("large", "fp64", 64) is None
    monkeypatch.setattr(bench, "PMC_SUMMARY", os.path.join(str(tmp_path), "missing.txt"))
    assert bench.stage_traffic("large", "fp64", 64) is None
