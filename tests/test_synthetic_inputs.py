"""The seeded input generators (synthetic/): loading histories of Sec. 4.1
(Eq. 27, the fully reversed cycles of the workloads and the R = 0 cycles
of Eq. 28 as intended) and the configurations."""

import numpy as np

from synthetic import config_by_name
from synthetic.loading import PERIOD, cyclic_history, macro_F


def test_macro_F_is_isochoric_and_uniaxial():
    for eps in (-0.01, 0.0, 0.006, 0.05):
        F = macro_F(eps)
        assert np.isclose(np.linalg.det(F), 1.0, rtol=1e-15)
        assert F[0, 0] == 1.0 + eps and F[1, 1] == F[2, 2]
        assert np.count_nonzero(F - np.diag(np.diag(F))) == 0


def test_r0_cycle_rises_to_the_peak_and_returns_to_zero():
    h = cyclic_history(0.01, 40, 3, kind="r0")
    assert len(h) == 120
    eps = np.array([i["eps"] for i in h])
    assert eps.min() >= 0.0 and np.isclose(eps.max(), 0.01, rtol=1e-15)
    for c in range(3):
        cyc = eps[40 * c: 40 * (c + 1)]
        assert np.isclose(cyc[19], 0.01, rtol=1e-15)       # t' = T/2
        assert cyc[-1] == 0.0                               # t' = T
        assert np.all(np.diff(cyc[:20]) > 0) and np.all(np.diff(cyc[19:]) < 0)
        # linear in time with slope 2 eps_max / T on the rise
        t = np.array([i["t"] for i in h[40 * c: 40 * c + 20]]) - c * PERIOD
        assert np.allclose(cyc[:20], 2 * 0.01 * t / PERIOD, rtol=1e-12)


def test_reversed_cycle_is_fully_reversed():
    eps = np.array([i["eps"] for i in cyclic_history(0.006, 40, 1)])
    assert np.isclose(eps.max(), 0.006) and np.isclose(eps.min(), -0.006)
    assert abs(eps[-1]) < 1e-18


def test_paper_workloads():
    for name, n, eps, cycles in (("P1_32", 32, 0.01, 3), ("P1_64", 64, 0.01, 3),
                                 ("P1_128", 128, 0.01, 3), ("P2", 64, 0.05, 3),
                                 ("P3", 32, 0.01, 100)):
        c = config_by_name(name)
        assert (c.n, c.eps_a, c.cycles, c.kind, c.grains) == (n, eps, cycles,
                                                             "r0", 235)
        h = c.history(cycles=1)
        assert min(i["eps"] for i in h) >= 0.0
    assert config_by_name("C3").kind == "reversed"
