"""Macroscopic deformation-gradient history of the cyclic strain test.

Sec. 4.1, Eq. 27: the applied macroscopic deformation gradient is isochoric
and nearly uniaxial, diag(F, F^{-1/2}, F^{-1/2}).  The stretch F(t) follows a
triangular cycle of period T = 4 s.  The printed cycle formula (Eq. 28) is
garbled; the workloads here are fully reversed (+eps_a / -eps_a) triangles
starting upward from zero, F = 1 + eps.  The R = 0 form the paper intends
(0 -> eps_max -> 0) is available as ``kind="r0"``.
"""

from __future__ import annotations

import numpy as np

PERIOD = 4.0  # s, Sec. 4.1


def macro_F(eps: float) -> np.ndarray:
    """Eq. 27 with F = 1 + eps; returned as a row-major 3x3 float64 array."""
    f = 1.0 + eps
    return np.diag([f, f ** -0.5, f ** -0.5]).astype(np.float64)


def triangle(s: float, kind: str = "reversed") -> float:
    """Normalised strain at cycle fraction s in [0, 1].

    ``reversed``: 0 -> +1 -> -1 -> 0 (4s, 2-4s, 4s-4).
    ``r0``:       0 -> +1 -> 0 (2s, 2-2s), the R = 0 cycle of Eq. 28.
    """
    if kind == "reversed":
        if s <= 0.25:
            return 4.0 * s
        if s <= 0.75:
            return 2.0 - 4.0 * s
        return 4.0 * s - 4.0
    if kind == "r0":
        return 2.0 * s if s <= 0.5 else 2.0 - 2.0 * s
    raise ValueError(f"unknown cycle kind {kind!r}")


def cyclic_history(eps_a: float, inc_per_cycle: int, cycles: int,
                   period: float = PERIOD, kind: str = "reversed"):
    """List of increments; each is a dict with the target macro F.

    Keys: ``k`` (1-based global increment), ``cycle`` (0-based), ``j``
    (1-based increment within the cycle), ``t``, ``dt``, ``eps``,
    ``F_bar`` (3x3), ``cycle_start`` (True for the first increment of a
    cycle) and ``cycle_end``.
    """
    dt = period / inc_per_cycle
    out = []
    k = 0
    for cyc in range(cycles):
        for j in range(1, inc_per_cycle + 1):
            k += 1
            s = j / inc_per_cycle
            eps = eps_a * triangle(s, kind)
            out.append(dict(k=k, cycle=cyc, j=j, t=k * dt, dt=dt, eps=eps,
                            F_bar=macro_F(eps), cycle_start=(j == 1),
                            cycle_end=(j == inc_per_cycle)))
    return out
