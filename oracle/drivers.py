"""Experiment drivers of App. A on top of the dense oracle MPO (FP64).

Test infrastructure only (see ``oracle/__init__``).

* EE-saturation stop rule (App. A, for the entropy-scaling figures): apply
  the interferometer layer by layer and stop once the largest bond entropy
  has not increased for ``patience`` (10 in the paper) consecutive layers, or
  when the layers run out; the quantity recorded is the maximum EE.  An
  "increase" is taken as exceeding the best value so far by more than
  ``1e-12`` bits (the paper gives no threshold; rounding must not count).
* Fixed-accuracy bond-dimension search (App. A, bond-dimension figure): run
  the whole interferometer at chi, double chi while 1 - Tr rho exceeds the
  target, then refine between the last failing and the first passing chi by
  bisection for a few more runs; the estimate is the smallest passing chi
  found.

Both take the circuit as layers of (k, theta, phi) and work on any object
with the DenseMPO interface, so the rules can also be checked on synthetic
entropy and error sequences.
"""
from __future__ import annotations

EE_EPS = 1e-12


def saturation_stop(layer_max_ee, patience: int = 10):
    """Apply the stop rule to per-layer maxima of the bond EE (an iterable,
    consumed lazily).  Returns (layers_used, best_ee, layer_of_best); layer
    indices are 1-based counts of applied layers, 0 = before any layer."""
    best, at, since, used = None, 0, 0, 0
    for s in layer_max_ee:
        used += 1
        if best is None or s > best + EE_EPS:
            best, at, since = s, used, 0
        else:
            since += 1
            if since >= patience:
                break
    return used, best, at


def run_until_saturation(mpo, layers, chi: int, patience: int = 10):
    """Dense-oracle run of the stop rule; returns (layers_used, S_max, layer_of_max)."""
    def per_layer():
        for layer in layers:
            for (k, th, ph) in layer:
                mpo.apply_gate(k, th, ph, chi)
            yield float(mpo.entropies().max())
    return saturation_stop(per_layer(), patience)


def chi_search(error_of, chi0: int, chi_max: int, target: float, refine: int):
    """Doubling then bisection on chi (App. A).  error_of(chi) -> 1 - Tr rho.
    Returns (chi_found or -1, its error, [(chi, error) in evaluation order])."""
    trials = []

    def err(c):
        e = float(error_of(c))
        trials.append((c, e))
        return e

    lo, chi = None, chi0
    e = err(chi)
    while e > target:
        if chi >= chi_max:
            return -1, e, trials
        lo = chi
        chi = min(2 * chi, chi_max)
        e = err(chi)
    hi, ehi = chi, e
    for _ in range(refine):
        if lo is None or hi - lo <= 1:
            break
        mid = (lo + hi) // 2
        em = err(mid)
        if em <= target:
            hi, ehi = mid, em
        else:
            lo = mid
    return hi, ehi, trials
