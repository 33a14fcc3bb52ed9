"""Solver-level parity of the HIP path with the CPU oracle (Sec. 2.1).

FP64 mode at a tight equilibrium tolerance (1e-12, CG 1e-10) reproduces
the oracle's fields to 1e-10 relative (max norm) at every increment; mixed
mode at 1e-6 matches the FP64 oracle's macroscopic loop to 1e-4 (Eq. 29)
and its fatigue indicator fields to 1e-3 (Eq. 30).  Also: homogeneous
medium, rollback of failed increments, bitwise checkpoint/resume, bitwise
determinism, graph-captured CG equal to direct launches.
"""

import numpy as np
import pytest

from gpu_util import make_rve, oracle_for, rel_maxnorm, to_soa
from synthetic import (config_by_name, macro_F, make_microstructure,
                       material_params)

pytestmark = pytest.mark.gpu

TIGHT = dict(newton_tol=1e-12, cg_tol=1e-10, newton_max_iter=40,
             cg_max_iter=5000)
ORACLE_TIGHT = dict(tol=1e-12, eta=1e-10, newton_max=40, cg_max=5000)


def _compare_state(r, o, tol=1e-10):
    """Every committed field the library exports against the oracle's."""
    got = r.fields("F", "P", "sigma", "Fpinv", "chi", "dgamma", "pcyc",
                   "pcyc_lit", "wcyc")
    ref = dict(F=to_soa(o.F), P=to_soa(o.P), sigma=to_soa(o.cauchy()),
               Fpinv=to_soa(o.Fpi), chi=o.chi.T, dgamma=o.dg.T, pcyc=o.pcyc,
               pcyc_lit=o.pcyc_lit, wcyc=o.wcyc.T)
    for k, v in ref.items():
        if np.max(np.abs(v)) < 1e-14:
            assert np.max(np.abs(got[k])) < 1e-14, k
        else:
            assert rel_maxnorm(got[k], v) < tol, k


def test_homogeneous_medium_single_evaluation():
    micro = make_microstructure(16, 1, 5)
    r = make_rve(micro, "continuous", **TIGHT)
    try:
        for eps in (0.002, 0.004):
            info = r.increment(macro_F(eps), 0.1)
            assert info["status"] == 0 and info["newton_iters"] == 0
            assert info["residuals"][0] < 1e-13
            F = r.field("F")
            assert np.max(np.abs(F - macro_F(eps).reshape(9, 1))) == 0.0
    finally:
        r.close()


# the whole C1 cycle is compared in test_gpu_vs_oracle.py; sched forces the
# CG matvec with the direction step and K:p folded into the first transform
# pass (one and three components per slab block)
@pytest.mark.parametrize("cfg,ninc,sched", [
    ("C1", 2, None), ("C2", 2, None), ("C1", 3, (1, 8, 1)),
    ("C1", 3, (3, 8, 1)), ("C2", 2, (1, 8, 1))])
def test_fp64_increments_match_oracle(cfg, ninc, sched):
    c = config_by_name(cfg)
    micro = c.microstructure()
    hist = c.history()[:ninc]
    r = make_rve(micro, c.operator, "fp64", **TIGHT)
    if sched:
        r.set_fft_schedule(*sched)
    o = oracle_for(micro, c.operator)
    try:
        for inc in hist:
            print(f"{cfg} increment {inc['k']} eps={inc['eps']:+.4f}", flush=True)
            info = r.increment(inc["F_bar"], inc["dt"])
            oi = o.increment(inc["F_bar"], inc["dt"], **ORACLE_TIGHT)
            assert info["status"] == 0 and oi.status == 0
            _compare_state(r, o)
            assert rel_maxnorm(info["P_bar"], oi.P_bar) < 1e-10
        if sched:
            assert r.fft_schedule()["fused"] == sched[2]
    finally:
        r.close()


def test_failed_increment_rolls_back_and_nan_is_local_failure():
    micro = config_by_name("C1").microstructure()
    r = make_rve(micro, "continuous", newton_max_iter=1)
    try:
        assert r.increment(macro_F(0.001), 0.2)["status"] in (0, -4)
        blob = r.get_state()
        fields = {k: r.field(k) for k in ("F", "P", "Fpinv", "chi", "pcyc")}
        info = r.increment(macro_F(0.03), 0.2)
        assert info["status"] == -4
        for k, v in fields.items():
            assert np.array_equal(r.field(k), v)
        assert r.get_state() == blob
        F = r.field("F")
        F[0, 17] = np.nan
        r.debug_set_field("F", F)
        info = r.increment(macro_F(0.002), 0.2)
        assert info["status"] == -5 and info["local_failures"] >= 1
        assert np.array_equal(r.field("Fpinv"), fields["Fpinv"])
    finally:
        r.close()


def test_checkpoint_resume_and_determinism_bitwise():
    c = config_by_name("C1")
    micro = c.microstructure()
    hist = c.history()[:6]
    a = make_rve(micro, c.operator)
    b = make_rve(micro, c.operator)
    try:
        for inc in hist[:3]:
            a.increment(inc["F_bar"], inc["dt"])
            b.increment(inc["F_bar"], inc["dt"])
        blob = a.get_state()
        assert blob == b.get_state()             # two runs, bitwise equal
        for inc in hist[3:]:
            a.increment(inc["F_bar"], inc["dt"])
        b.close()
        b = make_rve(micro, c.operator)
        b.set_state(blob)
        for inc in hist[3:]:
            b.increment(inc["F_bar"], inc["dt"])
        assert a.get_state() == b.get_state()   # resume is bitwise
    finally:
        a.close()
        b.close()


def test_graph_capture_equals_direct_launches():
    import torch
    c = config_by_name("C1")
    micro = c.microstructure()
    hist = c.history()[:3]
    s = torch.cuda.Stream()
    a = make_rve(micro, c.operator, "mixed", use_graph=False)
    b = make_rve(micro, c.operator, "mixed", use_graph=True, stream=s)
    try:
        for inc in hist:
            ia = a.increment(inc["F_bar"], inc["dt"])
            ib = b.increment(inc["F_bar"], inc["dt"])
            assert ia["status"] == ib["status"] == 0
            assert ia["residuals"] == ib["residuals"]
        assert a.get_state() == b.get_state()
    finally:
        a.close()
        b.close()


def test_cg_chunk_length_changes_only_where_the_host_checks():
    """The host checks CG convergence once per chunk (queued one ahead, the
    queued chunk sized from the observed r.r decay); the device iteration
    and its stopping decision do not depend on it: any chunk length gives
    the same bits."""
    c = config_by_name("C2")
    micro = c.microstructure()
    hist = c.history()[:3]
    runs = {}
    for chunk in (2, 8, 32):
        r = make_rve(micro, c.operator, "mixed", cg_chunk=chunk, cg_forcing=2)
        try:
            infos = [r.increment(inc["F_bar"], inc["dt"]) for inc in hist]
            assert all(i["status"] == 0 for i in infos)
            runs[chunk] = ([(i["cg_iters_total"], i["residuals"]) for i in infos],
                           r.get_state())
        finally:
            r.close()
    assert runs[2] == runs[8] == runs[32]


@pytest.mark.parametrize("graph", [False, True])
def test_live_kernel_timing_counts_and_leaves_results_unchanged(graph):
    """Live event timing brackets each launch of the chosen classes in the
    solver's own iteration (CG graphs included) and changes no result."""
    import torch
    from paper_1806_10599_amd.binding import KERNEL_CLASSES
    c = config_by_name("C1")
    micro = c.microstructure()
    hist = c.history()[:3]
    s = torch.cuda.Stream()
    a = make_rve(micro, c.operator, "mixed", use_graph=graph, stream=s)
    b = make_rve(micro, c.operator, "mixed", use_graph=graph, stream=s)
    try:
        b.set_kernel_timing(KERNEL_CLASSES)
        evals = cg = newton = 0
        for inc in hist:
            ia = a.increment(inc["F_bar"], inc["dt"])
            ib = b.increment(inc["F_bar"], inc["dt"])
            assert ia["status"] == ib["status"] == 0
            assert ia["residuals"] == ib["residuals"]
            evals += ib["newton_iters"] + 1
            newton += ib["newton_iters"]
            cg += ib["cg_iters_total"]
        assert a.get_state() == b.get_state()
        t = b.kernel_timing(reset=True)
        assert t["return_map"][1] == evals and t["residual_fp64"][1] == evals
        assert t["tangent"][1] == newton
        # launches past convergence: the rest of the converging chunk and
        # the chunk queued ahead of the host check (they return at once)
        chunk = 8
        fused = b.fft_schedule()["fused"]   # K:p inside pass A: no K:p kernel
        cgk = ("matvec_pass_a", "matvec_pass_b", "matvec_pass_c") + (
            () if fused else ("matvec_kp",))
        if fused:
            assert t["matvec_kp"] == (0.0, 0)
        for k in cgk:
            ms, n = t[k]
            assert ms > 0.0
            if graph:   # whole chunks are replayed
                assert n % chunk == 0 and cg <= n < cg + 2 * chunk * newton
            else:
                assert cg <= n < cg + 2 * chunk * newton
        assert all(v == (0.0, 0) for v in b.kernel_timing().values())
        cnt = b.return_map_counts(reset=True)
        assert cnt["crystal"] + cnt["particle"] == evals * micro.n ** 3
        assert cnt["evals"] >= cnt["crystal"] and cnt["steps"] >= 0
        b.set_kernel_timing(())
        inc = c.history()[3]
        ib = b.increment(inc["F_bar"], inc["dt"])
        ia = a.increment(inc["F_bar"], inc["dt"])
        assert ib["status"] == 0
        assert all(v == (0.0, 0) for v in b.kernel_timing().values())
        # one launch in seven of the CG classes: counted all, timed a sample
        b.set_kernel_timing(KERNEL_CLASSES, cg_stride=7)
        inc = c.history()[4]
        ib = b.increment(inc["F_bar"], inc["dt"])
        ia = a.increment(inc["F_bar"], inc["dt"])
        assert ib["residuals"] == ia["residuals"]
        t, seen = b.kernel_timing(), b.kernel_launches(reset=True)
        assert t["return_map"][1] == seen["return_map"] == ib["newton_iters"] + 1
        for k in cgk:
            if graph:   # replayed chunks time every launch (not counted)
                assert seen[k] == 0 and t[k][1] % 8 == 0 and t[k][1] > 0
            else:
                assert seen[k] >= ib["cg_iters_total"]
                assert t[k][1] == (seen[k] + 6) // 7 and t[k][0] > 0.0
        assert all(v == (0.0, 0) for v in b.kernel_timing().values())
    finally:
        a.close()
        b.close()


def test_fft_schedules_agree_and_autotune_picks_one():
    """Every valid CG-matvec schedule, with the direction step in its own
    kernel or folded into the first transform pass, gives the same
    increments (the schedules regroup the same per-component transforms;
    only the order of the p.Ap partial sums differs); the default tunes
    one."""
    from paper_1806_10599_amd.binding import RveError
    c = config_by_name("C1")
    micro = c.microstructure()
    hist = c.history()[:2]
    ref = make_rve(micro, c.operator, "mixed")
    try:
        ri = [ref.increment(inc["F_bar"], inc["dt"]) for inc in hist]
        sch = ref.fft_schedule()
        assert sch["cpb"] in (1, 3) and sch["tt"] in (4, 8, 16)
        assert sch["fused"] in (0, 1)
        assert sch["tuned_ms"] > 0.0
    finally:
        ref.close()
    for fused in (0, 1):
        for cpb in (1, 3):
            for tt in (4, 8, 16):
                r = make_rve(micro, c.operator, "mixed")
                try:
                    r.set_fft_schedule(cpb, tt, fused)
                    for inc, a in zip(hist, ri):
                        b = r.increment(inc["F_bar"], inc["dt"])
                        assert b["status"] == 0
                        assert b["newton_iters"] == a["newton_iters"]
                        assert rel_maxnorm(b["sigma_bar"], a["sigma_bar"]) < 1e-6
                    got = r.fft_schedule()
                    assert (got["cpb"], got["tt"], got["fused"]) == (cpb, tt, fused)
                    with pytest.raises(RveError):
                        r.set_fft_schedule(2, 8)
                    with pytest.raises(RveError):
                        r.set_fft_schedule(1, 8, 2)
                finally:
                    r.close()


def test_full_size_chosen_path_against_oracle(oracle_map):
    """The 64^3 workload (200 grains, 8 % particles, discrete operator) in
    the configuration bench.py times: mixed precision, learned start kept
    directly below half the homogeneous predictor's residual (warm_start 2),
    inexact-Newton forcing mode 2, CG chunks of 8.  After each of the first
    increments every voxel, grains and particles, is re-integrated by the
    oracle's point law from the previous committed state at the GPU's
    converged F (FP64 on both sides), and the whole-field conditions are
    checked with the oracle's projection: ||G(P)|| <= tol ||P|| (Sec. 2.1,
    Eq. 11) and F - F_bar compatible.  The mean <F> = F_bar holds to the
    FP32 rounding of the CG corrections: every CG iteration can shift the
    mean of its iterate by at most one FP32 rounding (2^-24) of the largest
    entry, so over an increment |<F> - F_bar| grows by at most
    (CG iterations) 2^-24 max|F - F_prev - dF_bar| (the corrections stay
    below the fluctuation increment in size; a factor 2 covers overshoot)."""
    import oracle_jobs
    from oracle.solver import OracleRVE
    from paper_1806_10599_amd.binding import Rve, WarmStartNet
    from paper_1806_10599_amd.warmstart import trained_params
    c = config_by_name("C3")
    micro = c.microstructure()
    hist = c.history()[:3]
    N = micro.n ** 3
    o = OracleRVE((micro.n,) * 3, micro.phase, micro.quat, micro.law,
                  material_params(), c.operator)
    net = WarmStartNet()
    net.set_params(trained_params())
    r = Rve(micro.n, projection=c.operator, precision="mixed", warm_start=2,
            cg_forcing=2, cg_chunk=8)
    r.set_microstructure(micro.phase, micro.quat, micro.law, material_params())
    r.attach_warm_start(net)
    chunks = np.array_split(np.arange(N), 12)
    try:
        prev = r.fields("F", "Fpinv", "chi")
        drift = np.zeros(9)
        Fb_prev = np.eye(3)
        for inc in hist:
            print(f"C3 increment {inc['k']}", flush=True)
            info = r.increment(inc["F_bar"], inc["dt"])
            assert info["status"] == 0 and info["residual_rel"] <= 1e-6
            got = r.fields("F", "P", "dgamma", "Fpinv", "chi")
            F = got["F"].T.reshape(N, 3, 3)
            P = got["P"].T.reshape(N, 3, 3)
            Fpi0 = prev["Fpinv"].T.reshape(N, 3, 3)
            chi0 = prev["chi"].T
            res = oracle_map(oracle_jobs.point_law, [
                (F[ix], Fpi0[ix], chi0[ix], micro.phase[ix], micro.quat,
                 micro.law, inc["dt"]) for ix in chunks])
            Pref = np.concatenate([x[0] for x in res])
            dgref = np.concatenate([x[1] for x in res])
            assert all(x[2].all() for x in res)
            err = np.max(np.abs(P - Pref)) / np.max(np.abs(Pref))
            derr = np.max(np.abs(got["dgamma"].T - dgref)) / max(
                np.max(np.abs(dgref)), 1e-300)
            print(f"  point law at all {N} voxels: P {err:.1e}, slips {derr:.1e}")
            assert err < 1e-9, err
            assert derr < 1e-9, derr
            # whole-field conditions with the oracle's projection
            resid = np.linalg.norm(o.G(P)) / np.linalg.norm(P)
            assert resid <= 1e-6 * (1 + 1e-6), resid
            Fb = np.asarray(inc["F_bar"]).reshape(3, 3)
            fl = F - Fb[None]
            comp = np.linalg.norm(o.G(fl) - fl) / np.linalg.norm(fl)
            assert comp < 1e-5, comp
            dfl = F - prev["F"].T.reshape(N, 3, 3) - (Fb - Fb_prev)[None]
            bound = info["cg_iters_total"] * 2.0 ** -24 * 2 * np.max(np.abs(dfl))
            step = (F.mean(axis=0) - Fb).reshape(9) - drift
            print(f"  <F> - F_bar grew by {np.max(np.abs(step)):.1e}"
                  f" (bound {bound:.1e})")
            assert np.max(np.abs(step)) <= bound
            drift = (F.mean(axis=0) - Fb).reshape(9)
            prev = {k: got[k] for k in ("F", "Fpinv", "chi")}
            Fb_prev = Fb
    finally:
        r.attach_warm_start(None)
        r.close()
        net.close()


def test_learned_form_at_128_validity(oracle_map):
    """The 128^3 workload (1000 grains, 5 % particles, discrete operator)
    in the benchmarked configuration (mixed precision, learned start kept
    directly, forcing mode 2, CG chunks of 8) over its first two increments
    (the second starts from the network).  After each, the oracle's point
    law at 16384 seeded voxels (grains and particles) from the GPU's
    converged F and the previous committed state; ||G(P)|| <= tol ||P||
    and F - F_bar compatible with the FP64 G of the library (compared
    element by element with the oracle's at 128^3 in
    test_apply_G_largest_grid_matches_oracle); <F> - F_bar within the FP32
    bound of test_full_size_chosen_path_against_oracle."""
    import oracle_jobs
    from paper_1806_10599_amd.binding import Rve, WarmStartNet
    from paper_1806_10599_amd.warmstart import trained_params
    c = config_by_name("C5")
    micro = c.microstructure()
    hist = c.history()[:2]
    N = micro.n ** 3
    law = micro.law[micro.phase]
    rng = np.random.default_rng(128)
    idx = np.sort(np.concatenate([
        rng.choice(np.nonzero(law == 0)[0], 14336, replace=False),
        rng.choice(np.nonzero(law == 1)[0], 2048, replace=False)]))
    chunks = np.array_split(idx, 8)
    net = WarmStartNet()
    net.set_params(trained_params())
    r = Rve(micro.n, projection=c.operator, precision="mixed", warm_start=2,
            cg_forcing=2, cg_chunk=8)
    r.set_microstructure(micro.phase, micro.quat, micro.law, material_params())
    r.attach_warm_start(net)
    try:
        prev = r.fields("F", "Fpinv", "chi")
        drift = np.zeros(9)
        Fb_prev = np.eye(3)
        for k, inc in enumerate(hist):
            print(f"C5 increment {inc['k']}", flush=True)
            info = r.increment(inc["F_bar"], inc["dt"])
            assert info["status"] == 0 and info["residual_rel"] <= 1e-6
            if k > 0:
                assert info["used_learned"] == 1
            got = r.fields("F", "P", "dgamma", "Fpinv", "chi")
            res = oracle_map(oracle_jobs.point_law, [
                (got["F"][:, ix].T.reshape(-1, 3, 3),
                 prev["Fpinv"][:, ix].T.reshape(-1, 3, 3), prev["chi"][:, ix].T,
                 micro.phase[ix], micro.quat, micro.law, inc["dt"])
                for ix in chunks])
            Pref = np.concatenate([x[0] for x in res]).reshape(-1, 9)
            dgref = np.concatenate([x[1] for x in res])
            assert all(x[2].all() for x in res)
            err = np.max(np.abs(got["P"][:, idx].T - Pref)) / np.max(np.abs(Pref))
            derr = np.max(np.abs(got["dgamma"][:, idx].T - dgref)) / max(
                np.max(np.abs(dgref)), 1e-300)
            print(f"  point law at {idx.size} voxels: P {err:.1e}, slips {derr:.1e}")
            assert err < 1e-9 and derr < 1e-9, (err, derr)
            P = got["P"]
            resid = np.linalg.norm(r.debug_apply_G(P)) / np.linalg.norm(P)
            assert resid <= 1e-6 * (1 + 1e-6), resid
            Fb = np.asarray(inc["F_bar"]).reshape(3, 3)
            fl = got["F"] - Fb.reshape(9, 1)
            comp = np.linalg.norm(r.debug_apply_G(fl) - fl) / np.linalg.norm(fl)
            assert comp < 1e-5, comp
            dfl = got["F"] - prev["F"] - (Fb - Fb_prev).reshape(9, 1)
            bound = info["cg_iters_total"] * 2.0 ** -24 * 2 * np.max(np.abs(dfl))
            step = (got["F"].mean(axis=1) - Fb.reshape(9)) - drift
            print(f"  ||G(P)||/||P|| {resid:.2e}, incompatibility {comp:.1e}, "
                  f"<F> - F_bar grew by {np.max(np.abs(step)):.1e} (bound {bound:.1e})")
            assert np.max(np.abs(step)) <= bound
            drift = got["F"].mean(axis=1) - Fb.reshape(9)
            prev = {key: got[key] for key in ("F", "Fpinv", "chi")}
            Fb_prev = Fb
    finally:
        r.attach_warm_start(None)
        r.close()
        net.close()


def test_cg_forcing_reaches_the_same_equilibrium_with_fewer_cg_iterations():
    """cg_forcing = 1 solves Newton iteration k only to
    min(0.1, max(cg_tol, newton_tol / (4 r_k))), cg_forcing = 2 to
    min(0.1, max(cg_tol, newton_tol / (2 r_k), 0.05 r_k)): every increment
    still ends at ||G(P)|| <= tol ||P||
    (FP64), the macroscopic stress agrees with the fixed-tolerance run to
    the equilibrium tolerance, and the CG count drops (mode 2 below
    mode 1)."""
    from paper_1806_10599_amd.binding import Rve
    c = config_by_name("C2")
    micro = c.microstructure()
    hist = c.history()[:12]
    runs = {}
    for forcing in (0, 1, 2):
        r = Rve(micro.n, projection=c.operator, precision="mixed",
                newton_tol=1e-6, cg_tol=1e-4, cg_forcing=forcing)
        r.set_microstructure(micro.phase, micro.quat, micro.law,
                             material_params())
        try:
            infos = []
            for inc in hist:
                info = r.increment(inc["F_bar"], inc["dt"])
                assert info["status"] == 0
                assert info["residual_rel"] <= 1e-6
                infos.append(info)
            runs[forcing] = infos
        finally:
            r.close()
    cg = {k: sum(i["cg_iters_total"] for i in v) for k, v in runs.items()}
    assert cg[1] < 0.95 * cg[0], cg
    assert cg[2] < cg[1], cg
    for mode in (1, 2):
        for a, b in zip(runs[0], runs[mode]):
            sa, sb = a["sigma_bar"][0, 0], b["sigma_bar"][0, 0]
            assert abs(sa - sb) <= 1e-5 * max(abs(sa), 1.0)


def test_extrapolated_start_reaches_the_same_equilibrium():
    """warm_start = 3 (the baseline the learned start is measured against):
    the last fluctuation increment scaled by the load ratio, projected by G
    and kept by the rule of warm_start = 2; every increment still ends at
    ||G(P)|| <= tol ||P|| and on the homogeneous-predictor run's macro
    stress to the equilibrium tolerance, and the extrapolation lowers the
    predictor residual away from load reversals."""
    from paper_1806_10599_amd.binding import Rve
    c = config_by_name("C2")
    micro = c.microstructure()
    hist = c.history()[:8]
    runs = {}
    for ws in (0, 3):
        r = Rve(micro.n, projection=c.operator, precision="mixed",
                newton_tol=1e-6, cg_tol=1e-4, cg_forcing=2, warm_start=ws)
        r.set_microstructure(micro.phase, micro.quat, micro.law,
                             material_params())
        try:
            infos = []
            for inc in hist:
                info = r.increment(inc["F_bar"], inc["dt"])
                assert info["status"] == 0 and info["residual_rel"] <= 1e-6
                infos.append(info)
            runs[ws] = infos
        finally:
            r.close()
    for a, b in zip(runs[0], runs[3]):
        sa, sb = a["sigma_bar"][0, 0], b["sigma_bar"][0, 0]
        assert abs(sa - sb) <= 1e-5 * max(abs(sa), 1.0)
    assert runs[3][0]["used_learned"] == 0         # no history yet
    used = [i["used_learned"] for i in runs[3][1:]]
    assert sum(used) >= len(used) - 1
    p0 = np.median([i["predictor_residual"] for i in runs[0][2:]])
    p3 = np.median([i["predictor_residual"] for i in runs[3][2:]])
    assert p3 < 0.5 * p0, (p3, p0)
