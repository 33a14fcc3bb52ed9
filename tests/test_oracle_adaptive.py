"""Pins of the oracle's automatic time incrementation
(OracleRVE.increment_adaptive): a converging step is a plain increment; a
cut step equals the plain increments at the fractions it reports; a step
that cannot be cut far enough leaves the state untouched."""

import numpy as np

from oracle.solver import OracleRVE, OK, ENOTCONV
from synthetic import macro_F, make_microstructure, material_params

KW = dict(tol=1e-8, eta=1e-10, cg_max=5000)


def _rve(n=6, grains=3, seed=7):
    m = make_microstructure(n, grains, seed)
    return OracleRVE((n,) * 3, m.phase, m.quat, m.law, material_params(),
                     "discrete")


def test_converging_step_is_a_plain_increment():
    a, b = _rve(), _rve()
    st, sub, cuts, steps = a.increment_adaptive(macro_F(0.002), 0.1,
                                                newton_max=25, **KW)
    info = b.increment(macro_F(0.002), 0.1, newton_max=25, **KW)
    assert st == OK and sub == 1 and cuts == 0
    assert np.array_equal(a.F, b.F) and np.array_equal(a.chi, b.chi)
    assert a.t == b.t == 0.1


def test_cut_step_equals_plain_increments_at_its_fractions():
    # three Newton corrections are not enough for the whole step
    a, b = _rve(), _rve()
    Fn = macro_F(0.006)
    st, sub, cuts, steps = a.increment_adaptive(Fn, 0.2, max_cutbacks=6,
                                                grow_after=2, newton_max=3,
                                                **KW)
    assert st == OK and cuts >= 1 and sub >= 2
    fr = [h for h, _ in steps]
    assert abs(sum(fr) - 1.0) == 0.0
    assert np.array_equal(a.F_bar, Fn)
    F0 = np.eye(3)
    done = 0.0
    for h, ia in steps:
        done += h
        tgt = Fn if done == 1.0 else F0 + done * (Fn - F0)
        ib = b.increment(tgt, h * 0.2, newton_max=3, **KW)
        assert ib.status == OK and ib.newton_iters == ia.newton_iters
    assert np.array_equal(a.F, b.F) and np.array_equal(a.pcyc, b.pcyc)
    assert np.isclose(a.t, 0.2, rtol=1e-15)


def test_growth_after_consecutive_successes():
    # without growth the sub-steps never lengthen; with growth after every
    # converged sub-step some do, and fewer sub-steps are needed
    runs = {}
    for g in (1, 10 ** 6):
        a = _rve()
        st, sub, cuts, steps = a.increment_adaptive(macro_F(0.006), 0.2,
                                                    max_cutbacks=8,
                                                    grow_after=g,
                                                    newton_max=3, **KW)
        assert st == OK and np.array_equal(a.F_bar, macro_F(0.006))
        runs[g] = [h for h, _ in steps]
    fixed = runs[10 ** 6]
    assert all(b <= a for a, b in zip(fixed, fixed[1:]))
    grow = runs[1]
    assert any(b > a for a, b in zip(grow, grow[1:]))
    assert len(grow) < len(fixed)


def test_exhausted_cutbacks_restore_the_state():
    a = _rve()
    a.increment(macro_F(0.001), 0.1, newton_max=25, **KW)
    before = {k: (v.copy() if isinstance(v, np.ndarray) else v)
              for k, v in a.__dict__.items()}
    st, sub, cuts, steps = a.increment_adaptive(macro_F(0.05), 0.1,
                                                max_cutbacks=1, newton_max=0,
                                                **KW)
    assert st == ENOTCONV and cuts == 2
    for k, v in before.items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(a.__dict__[k], v), k
        else:
            assert a.__dict__[k] == v, k
