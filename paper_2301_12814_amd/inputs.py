"""Seeded synthetic inputs (shared by tests, bench and smoke).

Holds no step of the method: only random numbers and the workload shapes.
The paper's workloads are synthetic too: Haar-random interferometers acting
on squeezed inputs with uniform loss (App. A).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def haar_unitary(M: int, seed: int) -> np.ndarray:
    """Haar-random M x M unitary: complex Ginibre -> QR -> fix column phases
    so that diag(R) is positive (Mezzadri's recipe)."""
    rng = np.random.default_rng(seed)
    Z = (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))) / math.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    ph = np.diag(R) / np.abs(np.diag(R))
    return Q * ph[None, :]


@dataclass
class Workload:
    name: str
    M: int
    r: list            # squeezing per mode (0 = vacuum)
    eta: float         # uniform transmission
    d: int             # per-mode Fock cutoff
    chi: int           # bond dimension
    seed: int          # Haar seed
    extra: dict = field(default_factory=dict)


def eta_sqrt_scaling(M: int, r: float) -> float:
    """Transmission with mean surviving photons eta*M*sinh^2 r = 2 sqrt(M sinh^2 r)."""
    return 2.0 / math.sqrt(M * math.sinh(r) ** 2)


def workload(name: str) -> Workload:
    if name == "small":          # M=8, d=4, chi=32: the oracle finishes in seconds
        return Workload("small", 8, [0.5] * 8, 0.5, 4, 32, 1)
    if name == "medium":         # M=32, r=0.8, eta from sqrt scaling, d=8, chi=256
        return Workload("medium", 32, [0.8] * 32, eta_sqrt_scaling(32, 0.8), 8, 256, 2)
    if name == "large":          # M=64, r=0.9, eta=0.3, d=8, chi=1024 (2016 gates)
        return Workload("large", 64, [0.9] * 64, 0.3, 8, 1024, 3)
    if name.startswith("table1"):
        # the shape of the paper's timing table (Sec. III.A): 12 modes, 10
        # squeezed inputs, photon loss 0.55 (transmission 0.45), d = 15 read as
        # a cap on the total photon number; r = 0.88 (about one photon per
        # squeezed mode, Sec. III.B) and the first 10 modes squeezed are
        # assumptions (the table states neither); "table1-<chi>" sets chi
        chi = int(name.split("-")[1]) if "-" in name else 1024
        return Workload(name, 12, [0.88] * 10 + [0.0] * 2, 0.45, 15, chi, 12,
                        extra={"total_cap": True})
    raise KeyError(name)


def batch_workloads(n: int = 256, base_seed: int = 1000):
    """The batched-instance law: M ~ U{16..48}, r ~ U[0.3, 1.2] (all modes),
    eta ~ U[0.2, 0.8], d ~ U{6, 8, 10}, chi ~ U{64, 128, 256, 512}; instance i
    seeded with base_seed + i (its Haar seed is the same number)."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(base_seed + i)
        M = int(rng.integers(16, 49))
        r = float(rng.uniform(0.3, 1.2))
        eta = float(rng.uniform(0.2, 0.8))
        d = int(rng.choice([6, 8, 10]))
        chi = int(rng.choice([64, 128, 256, 512]))
        out.append(Workload(f"batch{i}", M, [r] * M, eta, d, chi, base_seed + i))
    return out


LARGE_REQUEST = dict(M=96, r=1.0, eta=0.25, d=10, chi=1024)


def serving_requests(n: int, rate: float, seed: int = 5, p_large: float = 0.05,
                     base_seed: int = 5000):
    """Poisson request stream: exponential inter-arrival times at `rate`
    requests/s; each request follows the batched-instance law (Haar seed
    base_seed + i) or, with probability p_large, is the large request
    M=96, r=1.0, eta=0.25, d=10, chi=1024.  Returns [(arrival_s, Workload)]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        if rng.uniform() < p_large:
            L = LARGE_REQUEST
            w = Workload(f"req{i}-large", L["M"], [L["r"]] * L["M"], L["eta"], L["d"], L["chi"],
                         base_seed + i)
        else:
            w = batch_workloads(1, base_seed + i)[0]
            w.name = f"req{i}"
        out.append((t, w))
    return out
