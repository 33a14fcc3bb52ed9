"""Automatic time incrementation through the C ABI against the oracle's
(same reading): decisions (sub-steps, cutbacks, Newton corrections) and
fields in FP64; a converging step equals a plain increment bitwise; a step
that cannot be cut far enough restores the state bitwise (crystal and user
materials)."""

import numpy as np
import pytest

from gpu_util import rel_maxnorm, to_soa
from synthetic import macro_F, make_microstructure, material_params

pytestmark = pytest.mark.gpu

TOL = dict(newton_tol=1e-8, cg_tol=1e-10, cg_max_iter=5000)


def _rve(micro, newton_max, **kw):
    from paper_1806_10599_amd.binding import Rve
    r = Rve(micro.n, projection="discrete", precision="fp64",
            newton_max_iter=newton_max, **{**TOL, **kw})
    r.set_microstructure(micro.phase, micro.quat, micro.law, material_params())
    return r


def test_cutbacks_match_oracle():
    from oracle.solver import OracleRVE
    micro = make_microstructure(16, 4, 11)
    o = OracleRVE((16,) * 3, micro.phase, micro.quat, micro.law,
                  material_params(), "discrete")
    okw = dict(tol=1e-8, eta=1e-10, cg_max=5000)
    assert o.increment(macro_F(0.003), 0.1, newton_max=25, **okw).status == 0
    pre = _rve(micro, 25)
    r = _rve(micro, 3)
    try:
        assert pre.increment(macro_F(0.003), 0.1)["status"] == 0
        r.set_state(pre.get_state())
        print("adaptive step 0.3 % -> 0.5 %", flush=True)
        info = r.increment_adaptive(macro_F(0.005), 0.1, max_cutbacks=6,
                                    grow_after=2)
        st, sub, cuts, steps = o.increment_adaptive(macro_F(0.005), 0.1,
                                                    max_cutbacks=6,
                                                    grow_after=2,
                                                    newton_max=3, **okw)
        assert info["status"] == st == 0
        assert (info["substeps"], info["cutbacks"]) == (sub, cuts)
        assert cuts >= 1
        assert info["newton_iters_total"] == sum(i.newton_iters for _, i in steps)
        assert info["min_fraction"] == min(h for h, _ in steps)
        assert rel_maxnorm(r.field("F"), to_soa(o.F)) < 1e-10
        assert rel_maxnorm(r.field("pcyc"), o.pcyc) < 1e-9
        m = r.macro()
        assert np.array_equal(m["F_bar"], macro_F(0.005))
        assert abs(m["t"] - o.t) < 1e-15 and m["increments"] == o.increments
    finally:
        pre.close()
        r.close()


def test_converging_step_is_a_plain_increment():
    micro = make_microstructure(16, 4, 12)
    a, b = _rve(micro, 25), _rve(micro, 25)
    try:
        ia = a.increment_adaptive(macro_F(0.002), 0.1)
        ib = b.increment(macro_F(0.002), 0.1)
        assert ia["status"] == ib["status"] == 0
        assert ia["substeps"] == 1 and ia["cutbacks"] == 0
        assert ia["min_fraction"] == 1.0
        for f in ("F", "P", "chi", "pcyc", "wcyc"):
            assert np.array_equal(a.field(f), b.field(f)), f
    finally:
        a.close()
        b.close()


def test_exhausted_cutbacks_restore_the_state():
    micro = make_microstructure(16, 4, 13)
    pre = _rve(micro, 25)
    r = _rve(micro, 0)
    try:
        assert pre.increment(macro_F(0.002), 0.1)["status"] == 0
        r.set_state(pre.get_state())
        before = {f: r.field(f) for f in ("F", "P", "chi", "Fpinv", "pcyc",
                                           "wcyc", "dgamma")}
        m0 = r.macro()
        info = r.increment_adaptive(macro_F(0.006), 0.1, max_cutbacks=2)
        assert info["status"] == -4 and info["cutbacks"] == 3
        assert info["substeps"] == 0
        for f, v in before.items():
            assert np.array_equal(r.field(f), v), f
        m1 = r.macro()
        for k in ("F_bar", "P_bar", "t", "increments"):
            assert np.array_equal(m0[k], m1[k]), k
    finally:
        pre.close()
        r.close()


def test_exhausted_cutbacks_restore_user_material_state():
    from paper_1806_10599_amd.binding import Rve
    n = 16
    sv = np.stack([np.full(n ** 3, 80000.0), np.full(n ** 3, 120000.0),
                   np.zeros(n ** 3)])
    sv[0, : n ** 3 // 2] *= 6
    sv[1, : n ** 3 // 2] *= 6
    ok = Rve(n, projection="discrete", newton_tol=1e-10, cg_tol=1e-10,
             newton_max_iter=25)
    r = Rve(n, projection="discrete", newton_tol=1e-10, cg_tol=1e-10,
            newton_max_iter=1)
    try:
        ok.set_user_material("neo_hooke", sv)
        r.set_user_material("neo_hooke", sv)
        F1 = np.eye(3) + 0.02 * np.arange(9).reshape(3, 3) / 9
        assert ok.increment(F1, 0.1)["status"] == 0
        r.set_state(ok.get_state())
        s0, F0 = r.field("statev"), r.field("F")
        info = r.increment_adaptive(np.eye(3) + 0.2 * np.eye(3), 0.1,
                                    max_cutbacks=1)
        assert info["status"] == -4
        assert np.array_equal(r.field("statev"), s0)
        assert np.array_equal(r.field("F"), F0)
        # with enough corrections the same step converges on its own
        info = ok.increment_adaptive(np.eye(3) + 0.2 * np.eye(3), 0.1)
        assert info["status"] == 0
    finally:
        ok.close()
        r.close()


def test_bad_arguments():
    from paper_1806_10599_amd.binding import RveError
    micro = make_microstructure(16, 2, 14)
    r = _rve(micro, 25)
    try:
        for mc, ga in ((-1, 2), (31, 2), (4, 0)):
            with pytest.raises(RveError, match="RVE_EINVAL"):
                r.increment_adaptive(macro_F(0.001), 0.1, mc, ga)
        with pytest.raises(RveError, match="RVE_EINVAL"):
            r.increment_adaptive(macro_F(0.001), -0.1)
    finally:
        r.close()
