"""Kernel-level parity of the HIP library against the CPU oracle.

* G(A) (Sec. 2.1, Eq. 11) through the C ABI test hook, FP64 and FP32 FFT
  passes, both operators, every supported grid edge up to 96, a ragged
  (non-power-of-two) radix set (24 = 8*3, 40 = 8*5, 48 = 16*3, 96 = 8*4*3)
  and an anisotropic cell; at 128 (the largest grid) invariants instead.
* the point law and its tangent (Sec. 2.1, Eqs. 2 and 13; Sec. 3.2,
  Eq. 22) voxel by voxel against the oracle, at the initial state and at a
  non-trivial committed state, grains and particles mixed.
"""

import numpy as np
import pytest

from gpu_util import make_rve, rel_maxnorm
from oracle import crystal, material
from oracle.projection import apply_G
from synthetic import make_microstructure, material_params

pytestmark = pytest.mark.gpu


def _rve(n, op="discrete", **kw):
    from paper_1806_10599_amd.binding import Rve
    return Rve(n, projection=op, **kw)


@pytest.mark.parametrize("op", ["continuous", "discrete"])
@pytest.mark.parametrize("n", [16, 24, 32, 40, 48, 64, 96])
def test_apply_G_matches_oracle(n, op):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((9, n ** 3))
    ref = apply_G(A.reshape(3, 3, n, n, n), (1, 1, 1), op).reshape(9, -1)
    with _rve(n, op) as r:
        out64 = r.debug_apply_G(A, "fp64")
        out32 = r.debug_apply_G(A, "mixed")
    scale = np.max(np.abs(A))
    assert np.max(np.abs(out64 - ref)) < 1e-13 * scale
    assert np.max(np.abs(out32 - ref)) < 3e-6 * scale


def test_apply_G_anisotropic_cell():
    n, L = 32, (1.0, 2.0, 0.5)
    from paper_1806_10599_amd.binding import Rve
    rng = np.random.default_rng(3)
    A = rng.standard_normal((9, n ** 3))
    for op in ("continuous", "discrete"):
        ref = apply_G(A.reshape(3, 3, n, n, n), L, op).reshape(9, -1)
        with Rve(n, L=L, projection=op) as r:
            out = r.debug_apply_G(A, "fp64")
        assert np.max(np.abs(out - ref)) < 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("mixed", 3e-6)])
def test_apply_G_largest_grid_invariants(prec, tol):
    """128^3, both operators: G is idempotent, its output has zero mean, and
    a compatible single-mode field u = a sin(2 pi k.x) is reproduced, with
    grad u = a (x) v cos(2 pi k.x) for the operator's own wave vector:
    v = 2 pi k (continuous, Eq. 19) or v = n tan(pi k / n) (discrete,
    Eqs. 20-21, the rotated-difference gradient of a Fourier mode)."""
    n = 128
    rng = np.random.default_rng(128)
    A = rng.standard_normal((9, n ** 3))
    x = (np.arange(n) + 0.5) / n
    X = np.meshgrid(x, x, x, indexing="ij")
    k = np.array([3, -5, 7])
    arg = 2 * np.pi * (k[0] * X[0] + k[1] * X[1] + k[2] * X[2])
    a = np.array([0.3, -1.0, 0.7])
    for op in ("discrete", "continuous"):
        v = 2 * np.pi * k if op == "continuous" else n * np.tan(np.pi * k / n)
        comp = np.einsum("i,j,abc->ijabc", a, v, np.cos(arg)).reshape(9, -1)
        with _rve(n, op) as r:
            B = r.debug_apply_G(A, prec)
            BB = r.debug_apply_G(B, prec)
            out = r.debug_apply_G(comp, prec)
        assert np.max(np.abs(B.mean(axis=1))) < tol
        assert np.max(np.abs(BB - B)) < 10 * tol * np.max(np.abs(A))
        assert np.max(np.abs(out - comp)) < 10 * tol * np.max(np.abs(comp)), op
        if op == "discrete":   # the check tells the two operators apart
            vc = 2 * np.pi * k
            wrong = np.einsum("i,j,abc->ijabc", a, vc, np.cos(arg)).reshape(9, -1)
            assert np.max(np.abs(out - wrong)) > 1e-3 * np.max(np.abs(comp))


def _oracle_law(micro, F, Fpi0, chi0, dt):
    p = material_params()
    S0g, Cg = crystal.grain_tables(micro.quat, p)
    lam, mu = crystal.lame_from_young(p[8], p[9])
    N = F.shape[0]
    P = np.zeros((N, 3, 3))
    K = np.zeros((N, 3, 3, 3, 3))
    dg = np.zeros((N, 12))
    law = micro.law[micro.phase]
    cp = np.nonzero(law == 0)[0]
    el = np.nonzero(law == 1)[0]
    g = micro.phase[cp]
    out = material.cp_update(F[cp], Fpi0[cp], chi0[cp], np.zeros((cp.size, 12)),
                             S0g[g], Cg[g], p, dt)
    assert out["ok"].all()
    P[cp], K[cp], dg[cp] = out["P"], out["K"], out["dg"]
    if el.size:
        o2 = material.svk_update(F[el], lam, mu)
        P[el], K[el] = o2["P"], o2["K"]
    return P, K, dg


# FP32 tangent (mixed mode): the state is the FP64 one, the 6x6
# factorisation, the nine Woodbury solves and the assembly are FP32.  The
# max norm of K is set by its largest (elastic) entries, each assembled
# from a few tens of FP32 products and sums of terms no larger than itself,
# so its error stays within a few tens of unit roundoffs (2^-24) of the
# max norm: 32 x 2^-24 (measured up to 2.4e-7, four roundoffs)
K32_TOL = 32 * 2.0 ** -24


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("amp,state", [(6e-4, False), (3e-3, False),
                                       (3e-3, True)])
def test_constitutive_matches_oracle(amp, state, precision):
    """Return mapping (FP64 in both modes) and the tangent as the solver
    forms it (FP64, or FP32 linear algebra in mixed mode) at every voxel of
    a grain-and-particle RVE, against the oracle's point law."""
    micro = make_microstructure(16, 8, 77, particle_fraction=0.1)
    N = micro.n ** 3
    rng = np.random.default_rng(int(amp * 1e5) + state)
    F = np.eye(3) + amp * rng.standard_normal((N, 3, 3))
    Fpi0 = np.broadcast_to(np.eye(3), (N, 3, 3)).copy()
    chi0 = np.zeros((N, 12))
    r = make_rve(micro, precision=precision)
    try:
        if state:
            Fpi0 = Fpi0 + 1e-3 * rng.standard_normal((N, 3, 3))
            chi0 = 60.0 * np.tanh(rng.standard_normal((N, 12)))
            law = micro.law[micro.phase]
            Fpi0[law == 1] = np.eye(3)
            chi0[law == 1] = 0.0
            r.debug_set_field("Fpinv", Fpi0.reshape(N, 9).T)
            r.debug_set_field("chi", chi0.T)
        out = r.debug_constitutive(F.reshape(N, 9).T, 0.1)
    finally:
        r.close()
    assert out["fails"] == 0
    P, K, dg = _oracle_law(micro, F, Fpi0, chi0, 0.1)
    assert rel_maxnorm(out["P"], P.reshape(N, 9).T) < 1e-12
    eK = rel_maxnorm(out["K"], K.reshape(N, 81).T)
    print(f"{precision} amp {amp} state {state}: K max-norm error {eK:.2e}")
    assert eK < (1e-10 if precision == "fp64" else K32_TOL), eK
    assert np.max(np.abs(out["dg"] - dg.T)) < 1e-10 * max(np.max(np.abs(dg)), 1e-12) + 1e-17
