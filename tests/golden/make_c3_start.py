"""Writes c3_start.npz: the oracle's FP64 solution of the 64^3 workload
(200 grains, 8 % stiff particles, discrete operator of Eq. 21) over the
first three increments of its +-0.6 % cycles (40 per cycle), solved to an
equilibrium tolerance of 1e-9 (CG 1e-7): far below the 1e-4 (Eq. 29) and
1e-3 (Eq. 30) bars the mixed-precision path is held to against it.
Stored: P_bar, sigma_bar (Sec. 3.1) and the Newton count per increment, and
after the last increment F, P, P_cyc (both forms) and W_cyc at 4096 sampled
voxels.

Calls only the oracle and the seeded input generators (about an hour on
eight cores):
    python tests/golden/make_c3_start.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.solver import OracleRVE  # noqa: E402
from synthetic import config_by_name, material_params  # noqa: E402

NINC = 3
NSAMPLE = 4096
TOL, ETA = 1e-9, 1e-7
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_start.npz")


def main():
    c = config_by_name("C3")
    m = c.microstructure()
    hist = c.history()[:NINC]
    N = m.n ** 3
    idx = np.sort(np.random.default_rng(6464).choice(N, NSAMPLE, replace=False))
    o = OracleRVE((m.n,) * 3, m.phase, m.quat, m.law, material_params(),
                  c.operator)
    rec = dict(k=[], eps=[], P_bar=[], sigma_bar=[], newton=[])
    for inc in hist:
        oi = o.increment(inc["F_bar"], inc["dt"], tol=TOL, eta=ETA,
                         newton_max=40, cg_max=5000)
        assert oi.status == 0, (inc["k"], oi.status)
        print(f"increment {inc['k']} eps {inc['eps']:+.5f} newton "
              f"{oi.newton_iters} cg {oi.cg_iters_total}", flush=True)
        rec["k"].append(inc["k"])
        rec["eps"].append(inc["eps"])
        rec["P_bar"].append(oi.P_bar.reshape(9))
        rec["sigma_bar"].append(oi.sigma_bar.reshape(9))
        rec["newton"].append(oi.newton_iters)
    out = {k: np.asarray(v) for k, v in rec.items()}
    out.update(idx=idx, tol=TOL, eta=ETA, F=o.F[idx].reshape(-1, 9),
               P=o.P[idx].reshape(-1, 9), pcyc=o.pcyc[idx],
               pcyc_lit=o.pcyc_lit[idx], wcyc=o.wcyc[idx])
    np.savez(OUT, **out)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
