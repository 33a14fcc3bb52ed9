"""The benchmark workloads: sizes, grain counts, loading and material constants.

Five configurations, from the small oracle case to the large learned-start
case, and the paper's own histories (R = 0 cycles at 1 % on 32^3 to 128^3,
three cycles at 5 %, one hundred cycles at 1 %).  The material is the FCC power-law crystal with Armstrong-Frederick
back stress used by every workload (the paper's own Cruzado law is cited but
never written out, Sec. 3.2); particles are a stiff isotropic second phase
(Sec. 4.4).  Stresses and moduli in MPa, time in s.
"""

from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from .micro import make_microstructure, Microstructure
from .loading import cyclic_history

# Flat constant block passed across the C ABI (float64), in this order.
PARAM_NAMES = ("C11", "C12", "C44", "gdot0", "g", "n_exp", "c_af", "d_af",
               "E_particle", "nu_particle")


def material_params(C11=168400.0, C12=121400.0, C44=75400.0, gdot0=1e-3,
                    g=50.0, n_exp=20.0, c_af=20000.0, d_af=200.0,
                    E_particle=1.2e6, nu_particle=0.25) -> np.ndarray:
    return np.array([C11, C12, C44, gdot0, g, n_exp, c_af, d_af, E_particle,
                     nu_particle], dtype=np.float64)


@dataclass(frozen=True)
class RveConfig:
    name: str
    n: int
    grains: int
    particle_fraction: float
    operator: str            # "continuous" (Eq. 19) or "discrete" (Eq. 21)
    precision: str           # "fp64" or "mixed"
    eps_a: float
    inc_per_cycle: int
    cycles: int
    seed: int
    batch: int = 1           # RVEs in one batch (the batching workload)
    learned: bool = False
    kind: str = "reversed"   # cycle shape: "reversed" or "r0" (Eq. 28)

    @property
    def voxels(self) -> int:
        return self.n ** 3

    def microstructure(self) -> Microstructure:
        return make_microstructure(self.n, self.grains, self.seed,
                                   self.particle_fraction)

    def history(self, cycles: int | None = None):
        return cyclic_history(self.eps_a, self.inc_per_cycle,
                              self.cycles if cycles is None else cycles,
                              kind=self.kind)

    def batch_microstructures(self):
        """The batch of independent RVEs, each from its own seed.

        Per RVE j, from Generator(PCG64(seed + j)): grid edge uniform in
        {24, 32, 40, 48}, grain count uniform in [20, 150], then the usual
        draw order of ``make_microstructure``.
        """
        out = []
        for j in range(self.batch):
            rng = np.random.Generator(np.random.PCG64(self.seed + j))
            n = int(rng.choice([24, 32, 40, 48]))
            G = int(rng.integers(20, 151))
            out.append(make_microstructure(n, G, self.seed + j, 0.0, rng=rng))
        return out


CONFIGS = {
    "C1": RveConfig("C1", 16, 8, 0.0, "continuous", "fp64", 0.010, 20, 1, 1001),
    "C2": RveConfig("C2", 32, 64, 0.0, "discrete", "fp64", 0.008, 40, 3, 1002),
    "C3": RveConfig("C3", 64, 200, 0.08, "discrete", "mixed", 0.006, 40, 5, 1003),
    "C4": RveConfig("C4", 0, 0, 0.0, "discrete", "mixed", 0.005, 40, 10, 4000,
                    batch=32),
    "C5": RveConfig("C5", 128, 1000, 0.05, "discrete", "mixed", 0.005, 40, 10,
                    1005, learned=True),
    # the paper's own histories (Sec. 4.2, Sec. 5): R = 0 triangles of
    # period 4 s, 235 grains as in its RVE
    "P1_32": RveConfig("P1_32", 32, 235, 0.0, "discrete", "mixed", 0.01, 40,
                       3, 2032, kind="r0"),
    "P1_64": RveConfig("P1_64", 64, 235, 0.0, "discrete", "mixed", 0.01, 40,
                       3, 2064, kind="r0"),
    "P1_128": RveConfig("P1_128", 128, 235, 0.0, "discrete", "mixed", 0.01,
                        40, 3, 2128, kind="r0"),
    "P2": RveConfig("P2", 64, 235, 0.0, "discrete", "mixed", 0.05, 40, 3,
                    2264, kind="r0"),
    "P3": RveConfig("P3", 32, 235, 0.0, "discrete", "mixed", 0.01, 40, 100,
                    2332, kind="r0"),
}


def config_by_name(name: str, **overrides) -> RveConfig:
    cfg = CONFIGS[name]
    return replace(cfg, **overrides) if overrides else cfg
