"""Batched RVEs (one launch per pass for the whole batch) against the same
RVEs solved one by one through the single-RVE entry points, and per-RVE
convergence control.

The single-RVE path is itself pinned to the FP64 oracle (test_gpu_solver);
here the batch must reproduce it per RVE: in FP64 to 1e-10 (only the
summation order of the reductions differs), in mixed precision to the
mixed-precision bar (1e-4 on macro stress, Sec. 4, Eq. 29; 1e-3 on the
indicator fields, Eq. 30) against the FP64 single runs.
"""

import numpy as np
import pytest

from synthetic import config_by_name, make_microstructure, material_params

from gpu_util import make_rve, rel_maxnorm

pytestmark = pytest.mark.gpu


def _batch(micros, operator, precision, **kw):
    from paper_1806_10599_amd.binding import BatchRve
    b = BatchRve([m.n for m in micros], projection=operator,
                 precision=precision, **kw)
    for j, m in enumerate(micros):
        b.set_microstructure(j, m.phase, m.quat, m.law, material_params())
    return b


def _micros():
    # mixed edges, one RVE with particles (SVK law), several tile counts
    return [make_microstructure(16, 6, 11), make_microstructure(24, 10, 12),
            make_microstructure(32, 12, 13, 0.08),
            make_microstructure(16, 4, 14)]


def _run_single(micro, hist, operator, precision, **kw):
    r = make_rve(micro, operator, precision, **kw)
    try:
        out = []
        for inc in hist:
            if inc["cycle_start"]:
                r.reset_fips()
            out.append(r.increment(inc["F_bar"], inc["dt"]))
        fields = {k: r.field(k) for k in ("F", "P", "chi", "pcyc", "wcyc")}
        return out, fields, r.macro()
    finally:
        r.close()


@pytest.mark.parametrize("operator,forcing", [("continuous", 0),
                                              ("discrete", 0),
                                              ("discrete", 1),
                                              ("discrete", 2)])
def test_batch_fp64_matches_single_rves(operator, forcing):
    # with cg_forcing each RVE of the batch takes its own linear-solve
    # tolerances, the same as a single handle would
    micros = _micros()
    hist = config_by_name("C1").history()[:4]
    b = _batch(micros, operator, "fp64", cg_forcing=forcing)
    try:
        binfo = []
        for inc in hist:
            if inc["cycle_start"]:
                b.reset_fips()
            binfo.append(b.increment(inc["F_bar"], inc["dt"]))
        for j, m in enumerate(micros):
            sinfo, sf, smac = _run_single(m, hist, operator, "fp64",
                                          cg_forcing=forcing)
            for k in range(len(hist)):
                assert binfo[k][j]["status"] == 0
                assert binfo[k][j]["newton_iters"] == sinfo[k]["newton_iters"]
                assert abs(binfo[k][j]["cg_iters_total"]
                           - sinfo[k]["cg_iters_total"]) <= 2
                assert rel_maxnorm(binfo[k][j]["sigma_bar"],
                                   sinfo[k]["sigma_bar"]) < 1e-10
            for name, ref in sf.items():
                assert rel_maxnorm(b.field(j, name), ref) < 1e-10, (j, name)
            bm = b.macro(j)
            assert bm["increments"] == smac["increments"] == len(hist)
            assert abs(bm["t"] - smac["t"]) < 1e-12
    finally:
        b.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_mixed_meets_the_mixed_bar(graph):
    micros = _micros()[:3]
    hist = config_by_name("C1").history()[:4]
    b = _batch(micros, "discrete", "mixed", use_graph=graph)
    try:
        for inc in hist:
            infos = b.increment(inc["F_bar"], inc["dt"])
            assert all(i["status"] == 0 for i in infos)
            assert all(i["residual_rel"] <= 1e-6 for i in infos)
        for j, m in enumerate(micros):
            _, sf, smac = _run_single(m, hist, "discrete", "fp64")
            s_b, s_s = b.macro(j)["sigma_bar"], smac["sigma_bar"]
            assert np.max(np.abs(s_b - s_s)) <= 1e-4 * np.max(np.abs(s_s))
            pc = b.field(j, "pcyc")
            assert np.linalg.norm(pc - sf["pcyc"]) <= 1e-3 * np.linalg.norm(sf["pcyc"])
    finally:
        b.close()


def test_batch_per_rve_macro_and_retirement():
    """RVE 0 stays at F = I (zero stress: equilibrium at the predictor, no
    Newton step), RVE 1 is loaded; then with a Newton budget of one step
    the unloaded RVE commits while an overloaded one fails and keeps its
    committed state."""
    micros = _micros()[:2]
    hist = config_by_name("C1").history()
    I = np.eye(3)
    b = _batch(micros, "discrete", "fp64")
    try:
        for inc in hist[:2]:
            infos = b.increment(np.stack([I, inc["F_bar"]]), inc["dt"])
            assert [i["status"] for i in infos] == [0, 0]
            assert infos[0]["newton_iters"] == 0
            assert infos[0]["cg_iters_total"] == 0
            assert infos[1]["newton_iters"] >= 1
        assert b.macro(0)["increments"] == 2 and b.macro(1)["increments"] == 2
        np.testing.assert_array_equal(b.macro(1)["F_bar"], hist[1]["F_bar"])
        assert np.all(b.field(0, "P") == 0.0)
    finally:
        b.close()
    b = _batch(micros, "discrete", "fp64", newton_max_iter=1, newton_tol=1e-12)
    try:
        F_before = b.field(1, "F")
        F_big = 3.0 * hist[0]["F_bar"] - 2.0 * I
        infos = b.increment(np.stack([I, F_big]), hist[0]["dt"])
        assert infos[0]["status"] == 0 and infos[0]["newton_iters"] == 0
        assert infos[1]["status"] != 0
        assert b.macro(0)["increments"] == 1 and b.macro(1)["increments"] == 0
        np.testing.assert_array_equal(b.field(1, "F"), F_before)
    finally:
        b.close()


def test_batch_rejects_bad_input():
    from paper_1806_10599_amd.binding import BatchRve, RveError
    with pytest.raises(RveError):
        BatchRve([16, 96])          # 96 is not a batch edge
    m = make_microstructure(16, 4, 1)
    b = BatchRve([16, 16])
    try:
        b.set_microstructure(0, m.phase, m.quat, m.law, material_params())
        with pytest.raises(RveError):   # material constants differ
            b.set_microstructure(1, m.phase, m.quat, m.law,
                                 material_params(g=60.0))
        with pytest.raises(RveError):   # RVE 1 has no microstructure yet
            b.increment(np.eye(3), 0.1)
        with pytest.raises(RveError):
            b.macro(2)
    finally:
        b.close()


def test_c4_batch_workload_first_increment():
    """The 32-RVE mixed-edge batch workload: one increment converges for
    every RVE; two RVEs sampled against their single-RVE FP64 runs."""
    c = config_by_name("C4")
    micros = c.batch_microstructures()
    hist = c.history()
    b = _batch(micros, c.operator, c.precision, use_graph=True)
    try:
        infos = b.increment(hist[0]["F_bar"], hist[0]["dt"])
        assert all(i["status"] == 0 for i in infos)
        for j in (0, len(micros) - 1):
            _, _, smac = _run_single(micros[j], hist[:1], c.operator, "fp64")
            s_b, s_s = b.macro(j)["sigma_bar"], smac["sigma_bar"]
            assert np.max(np.abs(s_b - s_s)) <= 1e-4 * np.max(np.abs(s_s))
    finally:
        b.close()


@pytest.mark.parametrize("precision,forcing", [("fp64", 0), ("mixed", 2)])
def test_device_controlled_batch_equals_host_driven(precision, forcing):
    """use_graph: the Newton decisions taken on the device, each linear
    solve of every RVE in one persistent launch (grid barriers between the
    passes), the predictor and the first Newton iterations replayed from a
    captured graph.  The arithmetic is that of the host-driven batch, so
    the results are the same bits: statuses, Newton and CG counts, residual
    histories and every committed field."""
    micros = _micros()
    hist = config_by_name("C1").history()[:6]
    runs = []
    for graph in (False, True):
        b = _batch(micros, "discrete", precision, cg_forcing=forcing,
                   use_graph=graph)
        try:
            infos = []
            for inc in hist:
                if inc["cycle_start"]:
                    b.reset_fips()
                infos.append(b.increment(inc["F_bar"], inc["dt"]))
            fields = [{k: b.field(j, k) for k in ("F", "P", "chi", "pcyc",
                                                  "wcyc", "dgamma")}
                      for j in range(len(micros))]
            runs.append((infos, fields))
        finally:
            b.close()
    (ia, fa), (ib, fb) = runs
    for xa, xb in zip(ia, ib):
        for a, c in zip(xa, xb):
            assert a["status"] == c["status"] == 0
            for k in ("newton_iters", "cg_iters_total", "cg_iters",
                      "residuals"):
                assert a[k] == c[k], k
            assert np.array_equal(a["sigma_bar"], c["sigma_bar"])
    for da, db in zip(fa, fb):
        for k in da:
            assert np.array_equal(da[k], db[k]), k


def test_device_controlled_batch_past_the_captured_iterations():
    """A tight tolerance needs more Newton iterations than the captured
    graph holds: the rest run one at a time, the same bits as host-driven;
    and a Newton budget below the graph's iterations stops there."""
    micros = _micros()[:2]
    hist = config_by_name("C1").history()[:2]
    runs = []
    for graph in (False, True):
        b = _batch(micros, "discrete", "fp64", newton_tol=1e-12, cg_tol=1e-10,
                   newton_max_iter=40, cg_max_iter=5000, use_graph=graph)
        try:
            infos = [b.increment(inc["F_bar"], inc["dt"]) for inc in hist]
            runs.append((infos, [b.field(j, "F") for j in range(2)]))
        finally:
            b.close()
    (ia, fa), (ib, fb) = runs
    assert max(i["newton_iters"] for x in ib for i in x) > 4
    for xa, xb in zip(ia, ib):
        for a, c in zip(xa, xb):
            assert a["status"] == c["status"] == 0
            assert a["newton_iters"] == c["newton_iters"]
            assert a["residuals"] == c["residuals"]
    for a, c in zip(fa, fb):
        assert np.array_equal(a, c)
    b = _batch(micros, "discrete", "fp64", newton_tol=1e-12, cg_tol=1e-10,
               newton_max_iter=2, use_graph=True)
    try:
        infos = b.increment(hist[0]["F_bar"], hist[0]["dt"])
        assert all(i["status"] == -4 and i["newton_iters"] == 2 for i in infos)
        assert b.macro(0)["increments"] == 0
    finally:
        b.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_schedules_tuned_per_edge_and_forced_agree(graph):
    """Each grid edge of a batch gets its own CG-matvec schedule, tuned at
    the first increment (a valid one, with a positive tuned time) or
    forced; every forced combination gives the increments of the tuned
    batch (same Newton counts, sigma_bar to 1e-6: only the order of the
    p.Ap partial sums differs), on the host-driven and device-controlled
    paths.  Invalid schedules and edges are rejected; (0, 0) re-tunes."""
    from paper_1806_10599_amd.binding import RveError
    micros = _micros()[:2]          # edges 16 and 24
    hist = config_by_name("C1").history()[:2]
    ref = _batch(micros, "discrete", "mixed", use_graph=graph)
    try:
        ri = [ref.increment(inc["F_bar"], inc["dt"]) for inc in hist]
        sch = ref.fft_schedules()
        assert set(sch) == {16, 24}
        for e, s in sch.items():
            assert s["cpb"] in (1, 3) and s["tt"] in (4, 8, 16), (e, s)
            assert s["tuned_ms"] > 0.0
        sref = [ref.macro(j)["sigma_bar"] for j in range(2)]
    finally:
        ref.close()
    combos = [((1, 4), (3, 16)), ((3, 8), (1, 8)), ((1, 16), (3, 4))]
    for s16, s24 in combos:
        b = _batch(micros, "discrete", "mixed", use_graph=graph)
        try:
            b.set_fft_schedule(16, *s16)
            b.set_fft_schedule(24, *s24)
            for inc, a in zip(hist, ri):
                infos = b.increment(inc["F_bar"], inc["dt"])
                for i, ia in zip(infos, a):
                    assert i["status"] == 0
                    assert i["newton_iters"] == ia["newton_iters"]
            got = b.fft_schedules()
            assert (got[16]["cpb"], got[16]["tt"]) == s16
            assert (got[24]["cpb"], got[24]["tt"]) == s24
            assert got[16]["tuned_ms"] == 0.0
            for j in range(2):
                assert rel_maxnorm(b.macro(j)["sigma_bar"], sref[j]) < 1e-6
            with pytest.raises(RveError):
                b.set_fft_schedule(16, 2, 8)
            with pytest.raises(RveError):
                b.set_fft_schedule(32, 1, 8)
            b.set_fft_schedule(16, 0, 0)
            inc = config_by_name("C1").history()[2]
            assert all(i["status"] == 0
                       for i in b.increment(inc["F_bar"], inc["dt"]))
            assert b.fft_schedules()[16]["tuned_ms"] > 0.0
            assert (b.fft_schedules()[24]["cpb"],
                    b.fft_schedules()[24]["tt"]) == s24
        finally:
            b.close()
