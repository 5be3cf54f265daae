"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests
and the benchmark.

This module holds no arithmetic of the method: it only names the lattice
workloads (group, extents, coupling, flux, start, generator, seed) and draws
random run parameters.  Random numbers consumed by the method itself are
drawn by each side's own generator implementation from the same seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MRG32K3A, PHILOX, CONST = 0, 1, 2
COLD, HOT = 0, 1


@dataclass
class Workload:
    name: str
    group: int
    dims: tuple
    beta: float
    flux: int = 0
    start: int = HOT
    rng: int = PHILOX
    seed: int = 1
    nhit: int = 10
    n_hb: int = 1
    n_or: int = 0
    sweeps: int = 1
    lattice_id: int = 0

    @property
    def volume(self) -> int:
        return int(np.prod(self.dims))


# SU(2) 4^4, beta 2.3, cold start, MRG32k3a per-site streams from seed 1,
# ten heat-bath sweeps with the plaquette after each.
SU2_4x4 = Workload("su2_4^4_cold_mrg", 2, (4, 4, 4, 4), 2.3, start=COLD, rng=MRG32K3A,
                   seed=1, n_hb=1, n_or=0, sweeps=10)
# SU(3) 16^3x4 finite temperature, beta 5.69, Haar-random start (seed 7),
# 1 heat bath + 4 overrelaxation per compound sweep.
SU3_16x4 = Workload("su3_16^3x4_hot", 3, (16, 16, 16, 4), 5.69, start=HOT, rng=PHILOX,
                    seed=7, n_hb=1, n_or=4, sweeps=100)
# SU(3) 32^3x8, beta 5.9, lambda_3 background with n flux quanta, cold start.
def su3_32x8(flux: int = 0) -> Workload:
    return Workload(f"su3_32^3x8_n{flux}", 3, (32, 32, 32, 8), 5.9, flux=flux, start=COLD,
                    rng=PHILOX, seed=3, n_hb=1, n_or=4, sweeps=200)
# SU(3) 64^3x16, beta 6.0, hot start (seed 23).
SU3_64x16 = Workload("su3_64^3x16_hot", 3, (64, 64, 64, 16), 6.0, start=HOT, rng=PHILOX,
                     seed=23, n_hb=1, n_or=4, sweeps=50)


def batch_workloads(n: int = 64, seed: int = 11) -> list:
    """Independent lattices of uneven size: SU(2)/SU(3) 50/50, spatial extent
    uniform in {8,10,...,24}, temporal in {4,6}, beta uniform in [2.2,2.5]
    (SU(2)) or [5.5,6.0] (SU(3)); hot start, seed `seed`, lattice id = index."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(n):
        g = 2 if rng.random() < 0.5 else 3
        ns = int(rng.choice(np.arange(8, 25, 2)))
        nt = int(rng.choice([4, 6]))
        beta = float(rng.uniform(2.2, 2.5) if g == 2 else rng.uniform(5.5, 6.0))
        out.append(Workload(f"batch_{l}", g, (ns, ns, ns, nt), beta, start=HOT, rng=PHILOX,
                            seed=seed, n_hb=1, n_or=4, sweeps=50, lattice_id=l))
    return out


def random_params(seed: int, n: int):
    """Seeded scalar draws used by tests (e.g. coupling values)."""
    return np.random.default_rng(seed).random(n)
