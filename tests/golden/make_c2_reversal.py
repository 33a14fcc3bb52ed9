"""Writes c2_reversal.npz: the oracle's FP64 solution of the 32^3, 64-grain
polycrystal with the discrete operator (Eq. 21) over its first twelve
increments of +-0.8 % cycles (40 per cycle; the tenth is the first load
reversal, Eqs. 27-28 as fully reversed triangles), solved to an
equilibrium tolerance of 1e-12 (CG 1e-10).  Stored: the macroscopic stress
P_bar and sigma_bar (Sec. 3.1) and the Newton count at every increment,
F and P at 256 sampled voxels at every increment, and every state field at
those voxels after the last increment.

Calls only the oracle and the seeded input generators:
    python tests/golden/make_c2_reversal.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.solver import OracleRVE  # noqa: E402
from synthetic import config_by_name, material_params  # noqa: E402

NINC = 12
NSAMPLE = 256
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_reversal.npz")


def main():
    c = config_by_name("C2")
    m = c.microstructure()
    hist = c.history()[:NINC]
    N = m.n ** 3
    idx = np.sort(np.random.default_rng(2024).choice(N, NSAMPLE, replace=False))
    o = OracleRVE((m.n,) * 3, m.phase, m.quat, m.law, material_params(),
                  c.operator)
    rec = dict(k=[], eps=[], P_bar=[], sigma_bar=[], newton=[], F=[], P=[])
    for inc in hist:
        if inc["cycle_start"]:
            o.reset_fips()
        oi = o.increment(inc["F_bar"], inc["dt"], tol=1e-12, eta=1e-10,
                         newton_max=40, cg_max=5000)
        assert oi.status == 0, (inc["k"], oi.status)
        print(f"increment {inc['k']} eps {inc['eps']:+.4f} newton "
              f"{oi.newton_iters} cg {oi.cg_iters_total}", flush=True)
        rec["k"].append(inc["k"])
        rec["eps"].append(inc["eps"])
        rec["P_bar"].append(oi.P_bar.reshape(9))
        rec["sigma_bar"].append(oi.sigma_bar.reshape(9))
        rec["newton"].append(oi.newton_iters)
        rec["F"].append(o.F[idx].reshape(-1, 9))
        rec["P"].append(o.P[idx].reshape(-1, 9))
    out = {k: np.asarray(v) for k, v in rec.items()}
    out.update(idx=idx, Fpinv=o.Fpi[idx].reshape(-1, 9), chi=o.chi[idx],
               dgamma=o.dg[idx], pcyc=o.pcyc[idx], pcyc_lit=o.pcyc_lit[idx],
               wcyc=o.wcyc[idx], sigma=o.cauchy()[idx].reshape(-1, 9))
    np.savez(OUT, **out)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
