"""Pins of the App. A driver rules (oracle): the EE-saturation stop rule on
synthetic entropy sequences and the doubling-then-bisection bond-dimension
search on synthetic monotone error curves, against brute-force scans."""
import numpy as np
import pytest

from oracle import drivers


def test_stop_rule_on_synthetic_sequences():
    seq = [1.0, 2.0, 3.0, 3.0, 2.9, 3.0, 2.5]
    assert drivers.saturation_stop(seq, patience=2) == (5, 3.0, 3)
    assert drivers.saturation_stop(seq, patience=10) == (7, 3.0, 3)      # layers run out
    # a rise below the rounding threshold is not an increase
    assert drivers.saturation_stop([1.0, 1.0 + 1e-13, 1.0], patience=2) == (3, 1.0, 1)
    assert drivers.saturation_stop([1.0, 1.0 + 1e-9, 1.0], patience=2) == (3, 1.0 + 1e-9, 2)
    # the sequence is consumed lazily: nothing after the stop is evaluated
    seen = []

    def gen():
        for i, s in enumerate([5.0, 4.0, 4.0, 9.0, 9.0]):
            seen.append(i)
            yield s
    assert drivers.saturation_stop(gen(), patience=2) == (3, 5.0, 1)
    assert seen == [0, 1, 2]


@pytest.mark.parametrize("c_true", [1, 3, 17, 24, 100, 1000])
def test_chi_search_finds_the_smallest_passing_chi(c_true):
    err = lambda c: 1.0 / c if c < c_true else 0.001                  # noqa: E731
    target = 0.001
    brute = min(c for c in range(1, 2049) if err(c) <= target)
    got, e, trials = drivers.chi_search(err, 2, 2048, target, refine=20)
    if brute < 2:
        brute = 2
    assert got == brute and e == err(got)
    # doubling phase first: 2, 4, 8, ... up to the first pass
    k = 0
    while 2 * 2 ** k < brute:
        assert trials[k][0] == 2 * 2 ** k
        k += 1
    # every trial is scored with the error function
    assert all(t[1] == err(t[0]) for t in trials)


def test_chi_search_limited_refinement_and_failure():
    err = lambda c: 1.0 / c                                           # noqa: E731
    got, e, trials = drivers.chi_search(err, 1, 1024, 0.01, refine=1)
    assert got == 100 or (got >= 100 and err(got) <= 0.01)
    assert [t[0] for t in trials][:8] == [1, 2, 4, 8, 16, 32, 64, 128]
    assert trials[-1][0] == 96 and got == 128                          # one bisection step
    got, e, _ = drivers.chi_search(err, 1, 64, 0.001, refine=3)
    assert got == -1 and e == err(64)
