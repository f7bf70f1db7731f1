"""Driven-cavity workloads (Sec. 5.1) used by the tests and the benchmark.

Each preset states the spatial grid, velocity grid, Knudsen number
(delta = 1/Kn), lid velocity (units of V0 = sqrt(2 k T0 / m)), deviation scale
eps (= lid amplitude), Monte Carlo pairs per cell per step, CFL number, step
count and the uniform share of the pair law (a quarter: the Maxwellian law
alone is mean-square unstable at these time steps).  Values only: no part of
the method is computed here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace


@dataclass(frozen=True)
class Preset:
    name: str
    nx: int
    ny: int
    nv: int
    vmax: float
    kn: float
    lid_u: float
    eps: float
    n_pairs: int
    steps: int
    cfl: float = 0.5
    order: int = 2
    seed: int = 1
    sample_group: int = 1
    mix16: int = 4               # uniform share of the node-pair law, in 1/16
    lid_omega: float = 0.0       # lid_u * sin(lid_omega * t) when > 0
    moments_every: int = 0
    rv: float = 0.0              # velocity cells stretched in this ratio (0: uniform)
    continuous: bool = False     # pairs from the continuous Maxwellian (Box-Muller), binned to cells
    sequential: bool = False     # collision in place, sample after sample (Alg. 3)
    rx: float = 0.0              # spatial cells stretched in these ratios (0: uniform; order 1)
    ry: float = 0.0

    @property
    def delta(self) -> float:
        return 1.0 / self.kn

    def problem(self, **over) -> dict:
        kw = dict(nx=self.nx, ny=self.ny, nv=self.nv, vmax=self.vmax, delta=self.delta, eps=self.eps,
                  n_pairs=self.n_pairs, cfl=self.cfl, order=self.order, seed=self.seed,
                  sample_group=self.sample_group, mix16=self.mix16, rv=self.rv, rx=self.rx, ry=self.ry)
        flags = (4 if self.continuous else 0) | (8 if self.sequential else 0)
        if flags:
            kw["flags"] = flags  # BOLTZ_CONTINUOUS_PAIRS | BOLTZ_SEQUENTIAL_UPDATE
        kw.update(over)
        return kw

    def lid(self, t: float) -> float:
        """Lid velocity at the start time t of a step."""
        if self.lid_omega > 0.0:
            return self.lid_u * math.sin(self.lid_omega * t)
        return self.lid_u

    def with_(self, **over) -> "Preset":
        return replace(self, **over)


# 16x16 cells, 12^3 on [-4.5, 4.5], Kn = 0.1, lid 0.1, 2000 pairs, 50 steps
CAVITY_16 = Preset("cavity 16x16, 12^3 velocities, Kn 0.1, 2000 pairs/cell", 16, 16, 12, 4.5, 0.1, 0.1, 0.1,
                   2000, 50)
# 64x64 cells, 20^3 on [-5, 5], Kn = 0.05, lid 0.1, 20000 pairs, 1000 steps
CAVITY_64 = Preset("cavity 64x64, 20^3 velocities, Kn 0.05, 20000 pairs/cell", 64, 64, 20, 5.0, 0.05, 0.1, 0.1,
                   20000, 1000)
# 200x200 cells, 24^3 on [-5, 5], Kn = 0.01, lid 0.05 sin(0.5 t), 50000 pairs, 2000 steps
CAVITY_200 = Preset("cavity 200x200, 24^3 velocities, Kn 0.01, 50000 pairs/cell, oscillating lid", 200, 200, 24,
                    5.0, 0.01, 0.05, 0.05, 50000, 2000, lid_omega=0.5, moments_every=10)

# The paper's own benchmark discretisation (Sec. 5.1): delta = 1, 160x160
# cells (N_r = 25600), 20^3 velocity cells on [-3, 3] stretched in the ratio
# 0.945, N_t = 6144, lid velocity 0.01, CFL 0.5
CAVITY_PAPER = Preset("cavity 160x160, 20^3 velocities stretched 0.945 on [-3, 3], delta 1, 6144 pairs/cell "
                      "from the continuous Maxwellian (Box-Muller)",
                      160, 160, 20, 3.0, 1.0, 0.01, 0.01, 6144, 1000, rv=0.945, continuous=True)

# The same with every paper-literal option (Sec. 3, 4, 5.1): first-order
# streaming (Eq. streaming2D) on spatial cells stretched 0.996 (x) and 0.998
# (y), smallest at the side walls and the lid, and the in-place sequential
# collision of Alg. 3
CAVITY_PAPER_LITERAL = CAVITY_PAPER.with_(
    name="cavity 160x160, spatial cells stretched 0.996 / 0.998, first-order streaming, 20^3 velocities stretched "
         "0.945 on [-3, 3], delta 1, 6144 pairs/cell from the continuous Maxwellian, in-place sequential collision",
    order=1, rx=0.996, ry=0.998, sequential=True, sample_group=0)

PRESETS = {"cavity16": CAVITY_16, "cavity64": CAVITY_64, "cavity200": CAVITY_200, "paper160": CAVITY_PAPER,
           "paper160_literal": CAVITY_PAPER_LITERAL}
