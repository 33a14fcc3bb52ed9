"""Oracle runs that the GPU parity tests compare against (not collected).

Each job solves a load history with the CPU oracle in FP64 at a tight
equilibrium tolerance (1e-12, CG 1e-10, Sec. 2.1) and returns, per
increment, the state fields and the macroscopic stress.  The jobs are
independent of each other and of the GPU: `conftest.py` starts the ones the
selected tests need in worker processes when collection ends, so that they
run while the GPU tests before them do.

Histories (all on grids the oracle solves in seconds per increment):
* c1_cycle: the 16^3, 8-grain polycrystal with the continuous operator
  (Eq. 19) over its whole +-1 % cycle (20 increments, Eqs. 27-28 as fully
  reversed triangles) and the first increment of a second cycle, which
  starts with zero indicator accumulators (Sec. 3.3).
* c1_shear: the same microstructure under a non-diagonal, non-symmetric
  macroscopic deformation gradient (three increments), where sigma_bar =
  P_bar F_bar^T / det F_bar (Sec. 3.1) is sensitive to a transposition.
* c1_r0: the same microstructure under the R = 0 cycle the paper applies
  (0 -> 1 % -> 0, Sec. 4.1, Eq. 28 as intended), past its peak.
* adapt5: a 16^3, 8-grain polycrystal under the 5 % R = 0 cycle of Sec. 4.2
  with automatic time incrementation (a Newton budget of four corrections
  makes every whole increment fail and its halves converge).
* batch16 / batch24: two RVEs of the mixed-edge batch test.
* g128_discrete / g128_continuous: G (Eq. 11) of a seeded random field on
  the 128^3 grid (the largest one) with either operator.
"""

from __future__ import annotations

import os

import numpy as np

WORKERS = 6
TIGHT = dict(tol=1e-12, eta=1e-10, newton_max=40, cg_max=5000)
ADAPT = dict(tol=1e-8, eta=1e-10, newton_max=4, cg_max=5000)

# non-diagonal, non-symmetric macroscopic increment per step (det > 0)
SHEAR_STEP = np.array([[1.0e-3, 2.5e-3, 0.0],
                       [0.0, -5.0e-4, 1.0e-3],
                       [5.0e-4, 0.0, -5.0e-4]])


def shear_history(steps=3, dt=0.2):
    return [dict(k=k, F_bar=np.eye(3) + k * SHEAR_STEP, dt=dt,
                 cycle_start=(k == 1)) for k in range(1, steps + 1)]


def c1_micro():
    from synthetic import config_by_name
    return config_by_name("C1").microstructure()


def c1_cycle_history():
    from synthetic import config_by_name
    return config_by_name("C1").history(cycles=2)[:21]


def r0_history():
    from synthetic.loading import cyclic_history
    return cyclic_history(0.01, 20, 1, kind="r0")[:12]


def adapt5_micro():
    from synthetic import make_microstructure
    return make_microstructure(16, 8, 2016)


def adapt5_history():
    from synthetic import config_by_name
    return config_by_name("P2").history()[:3]


def batch_micros():
    from synthetic import make_microstructure
    return [make_microstructure(16, 6, 21), make_microstructure(24, 10, 22)]


def batch_history():
    from synthetic import config_by_name
    return config_by_name("C1").history()[:5]


def _oracle(micro, operator):
    from oracle.solver import OracleRVE
    from synthetic import material_params
    return OracleRVE((micro.n,) * 3, micro.phase, micro.quat, micro.law,
                     material_params(), operator)


def _snapshot(o, info=None):
    N = o.N
    s = dict(F=o.F.reshape(N, 9).T.copy(), P=o.P.reshape(N, 9).T.copy(),
             Fpinv=o.Fpi.reshape(N, 9).T.copy(), chi=o.chi.T.copy(),
             dgamma=o.dg.T.copy(), pcyc=o.pcyc.copy(),
             pcyc_lit=o.pcyc_lit.copy(), wcyc=o.wcyc.T.copy(),
             sigma=o.cauchy().reshape(N, 9).T.copy(),
             F_bar=o.F_bar.copy(), t=o.t, increments=o.increments)
    if info is not None:
        s.update(P_bar=info.P_bar.copy(), sigma_bar=info.sigma_bar.copy(),
                 newton=info.newton_iters, status=info.status)
    return s


def _history(micro, operator, hist):
    o = _oracle(micro, operator)
    out = []
    for inc in hist:
        if inc.get("cycle_start"):
            o.reset_fips()
        info = o.increment(inc["F_bar"], inc["dt"], **TIGHT)
        assert info.status == 0, (inc, info.status)
        out.append(_snapshot(o, info))
    return out


def job_c1_cycle():
    return _history(c1_micro(), "continuous", c1_cycle_history())


def job_c1_shear():
    return _history(c1_micro(), "continuous", shear_history())


def job_c1_r0():
    return _history(c1_micro(), "continuous", r0_history())


def job_adapt5():
    o = _oracle(adapt5_micro(), "discrete")
    out = []
    for inc in adapt5_history():
        st, sub, cuts, steps = o.increment_adaptive(
            inc["F_bar"], inc["dt"], max_cutbacks=6, grow_after=2, **ADAPT)
        assert st == 0, (inc["k"], st)
        s = _snapshot(o)
        s.update(substeps=sub, cutbacks=cuts,
                 newton_total=sum(i.newton_iters for _, i in steps),
                 min_fraction=min(h for h, _ in steps),
                 last_sigma_bar=steps[-1][1].sigma_bar.copy())
        out.append(s)
    return out


def job_batch16():
    return _history(batch_micros()[0], "discrete", batch_history())


def job_batch24():
    return _history(batch_micros()[1], "discrete", batch_history())


def g128_input():
    n = 128
    return np.random.default_rng(128).standard_normal((9, n ** 3))


def _g128(operator):
    from oracle.projection import apply_G
    n = 128
    return apply_G(g128_input().reshape(3, 3, n, n, n), (1.0, 1.0, 1.0),
                   operator).reshape(9, -1)


def job_g128_discrete():
    return _g128("discrete")


def job_g128_continuous():
    return _g128("continuous")


# longest first
JOBS = {
    "c1_cycle": job_c1_cycle,
    "g128_discrete": job_g128_discrete,
    "g128_continuous": job_g128_continuous,
    "c1_r0": job_c1_r0,
    "batch24": job_batch24,
    "adapt5": job_adapt5,
    "batch16": job_batch16,
    "c1_shear": job_c1_shear,
}


def point_law(args):
    """The oracle's point law (Sec. 2.1, Eq. 2; Sec. 3.2, Eq. 22) at given
    F (n, 3, 3) from a committed state (Fp^-1 (n, 3, 3), chi (n, 12)) for
    voxels of the given labels: returns (P, slips, ok)."""
    from oracle import crystal, material
    from synthetic import material_params
    F, Fpi0, chi0, label, quat, law, dt = args
    p = material_params()
    S0g, Cg = crystal.grain_tables(quat, p)
    lam, mu = crystal.lame_from_young(p[8], p[9])
    n = F.shape[0]
    P = np.zeros((n, 3, 3))
    dg = np.zeros((n, 12))
    ok = np.ones(n, dtype=bool)
    cp = np.nonzero(law[label] == 0)[0]
    el = np.nonzero(law[label] == 1)[0]
    if cp.size:
        g = label[cp]
        out = material.cp_update(F[cp], Fpi0[cp], chi0[cp],
                                 np.zeros((cp.size, 12)), S0g[g], Cg[g], p, dt,
                                 tangent=False)
        P[cp], dg[cp], ok[cp] = out["P"], out["dg"], out["ok"]
    if el.size:
        P[el] = material.svk_update(F[el], lam, mu, False)["P"]
    return P, dg, ok


def run(name):
    return JOBS[name]()


def worker_init():
    # a few BLAS threads per worker: the workers run side by side
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "2"
