"""Pins of the oracle's Newton-CG increment (CPU only).

* homogeneous medium: F = Fbar exactly, one constitutive evaluation, no CG;
* laminate: the exact discrete solution is piecewise constant with traction
  continuity across the layers (solved here as a 3-unknown problem);
* dense brute force on 4^3 and 5^3: Newton with dense least-squares linear
  steps (5^3 with the operator built from the textbook Fourier
  differentiation matrix) against Newton-CG;
* directional finite differences of G(P(F)) against G(K : v);
* <F> = Fbar, Hill-Mandel at convergence, quadratic Newton convergence;
* single-crystal fatigue indicators in closed form from the scalar law;
* failed increments leave the committed state untouched.
"""

import numpy as np
import pytest

from oracle import crystal, material
from oracle.solver import OracleRVE, OK, ENOTCONV, ELOCAL
from oracle.projection import dense_G
from synthetic import material_params, macro_F, shoemake_quaternions
from test_oracle_material import scalar_single_crystal_step
from test_oracle_projection import fourier_diff_matrix, gradient_matrix, \
    range_projector

P = material_params()
RNG = np.random.default_rng(99)
TIGHT = dict(tol=1e-12, eta=1e-12, newton_max=40, cg_max=5000)


def rve_from_labels(n, labels, quats, laws=None, operator="continuous"):
    laws = np.zeros(len(quats), dtype=np.int32) if laws is None else laws
    return OracleRVE((n, n, n) if np.isscalar(n) else n, labels, quats, laws,
                     P, operator)


def test_homogeneous_single_grain_one_evaluation():
    n = 6
    q = shoemake_quaternions(RNG.random((1, 3)))
    rve = rve_from_labels(n, np.zeros(n ** 3, dtype=np.int32), q)
    for eps in (0.003, 0.006, 0.002):
        info = rve.increment(macro_F(eps), 0.1, **TIGHT)
        assert info.status == OK
        assert info.newton_iters == 0 and info.cg_iters_total == 0
        assert info.residuals[0] < 1e-14
        assert np.max(np.abs(rve.F - macro_F(eps))) == 0.0


def test_single_crystal_fips_closed_form():
    n = 4
    rve = rve_from_labels(n, np.zeros(n ** 3, dtype=np.int32),
                          np.array([[1.0, 0, 0, 0]]))
    p1 = p2 = 1.0
    chis = 0.0
    pc = plit = w = 0.0
    for eps in (0.003, 0.006, 0.003, 0.0):
        info = rve.increment(macro_F(eps), 0.1, **TIGHT)
        assert info.status == OK
        dgam, st = scalar_single_crystal_step(1 + eps, p1, p2, chis, 0.1, P)
        p1, p2, chis = st["p1"], st["p2"], st["chi"]
        # dLp = dgam diag(8, -4, -4) / sqrt(6): dLp:dLp = 16 dgam^2
        pc += np.sqrt(32.0 / 3.0) * abs(dgam)       # sqrt(2/3 dLp:dLp)
        plit += 16.0 * dgam ** 2 / 0.1              # Eq. 23 integrand x dt
        w += st["tau"] * dgam
        assert np.allclose(rve.pcyc, pc, rtol=1e-9, atol=1e-15)
        assert np.allclose(rve.pcyc_lit, plit, rtol=1e-9, atol=1e-18)
        wa = rve.wcyc[:, np.abs(rve.dg[0]) > 1e-12]
        assert wa.shape[1] == 8
        assert np.allclose(wa, w, rtol=1e-8, atol=1e-12)
        assert np.isclose(info.P_bar[0, 0], st["P1"], rtol=1e-10)
    assert plit > 0.0   # the history does yield
    # a new cycle starts from zero accumulators (reading: per-cycle sums)
    rve.reset_fips()
    info = rve.increment(macro_F(0.003), 0.1, **TIGHT)
    assert info.status == OK
    dgam, st = scalar_single_crystal_step(1.003, p1, p2, chis, 0.1, P)
    assert np.allclose(rve.pcyc, np.sqrt(32.0 / 3.0) * abs(dgam), rtol=1e-9,
                       atol=1e-15)
    assert np.allclose(rve.pcyc_lit, 16.0 * dgam ** 2 / 0.1, rtol=1e-9,
                       atol=1e-18)


def _laminate_reference(rveA_q, lawA, lawB, history, phiA):
    """Exact discrete laminate: F_A = Fb + phiB c e1, F_B = Fb - phiA c e1."""
    phiB = 1 - phiA
    states = [dict(Fpi=np.eye(3)[None], chi=np.zeros((1, 12))) for _ in "AB"]
    S0, C = crystal.grain_tables(rveA_q, P)
    lam, mu = crystal.lame_from_young(P[8], P[9])

    def law(k, Fx, st, dt):
        kind = (lawA, lawB)[k]
        if kind == 1:
            return material.svk_update(Fx[None], lam, mu, False)["P"][0], st
        out = material.cp_update(Fx[None], st["Fpi"], st["chi"],
                                 np.zeros((1, 12)), S0[k:k + 1], C[k:k + 1],
                                 P, dt, tangent=False)
        return out["P"][0], dict(Fpi=out["Fpi"], chi=out["chi"])

    c = np.zeros(3)
    e1 = np.array([1.0, 0, 0])
    out = []
    for Fb, dt in history:
        for _ in range(60):
            FA = Fb + phiB * np.outer(c, e1)
            FB = Fb - phiA * np.outer(c, e1)
            r = law(0, FA, states[0], dt)[0][:, 0] - law(1, FB, states[1],
                                                        dt)[0][:, 0]
            if np.max(np.abs(r)) < 1e-11:
                break
            J = np.zeros((3, 3))
            h = 1e-7
            for j in range(3):
                dc = np.zeros(3)
                dc[j] = h
                rp = (law(0, Fb + phiB * np.outer(c + dc, e1), states[0], dt)
                      [0][:, 0] - law(1, Fb - phiA * np.outer(c + dc, e1),
                                      states[1], dt)[0][:, 0])
                J[:, j] = (rp - r) / h
            c = c - np.linalg.solve(J, r)
        FA = Fb + phiB * np.outer(c, e1)
        FB = Fb - phiA * np.outer(c, e1)
        _, states[0] = law(0, FA, states[0], dt)
        _, states[1] = law(1, FB, states[1], dt)
        out.append((FA, FB))
    return out


@pytest.mark.parametrize("op", ["continuous", "discrete"])
@pytest.mark.parametrize("lawB", [0, 1])
def test_laminate_exact_solution(op, lawB):
    n = 16                               # 8 | 8 split: no Nyquist content
    labels = np.zeros((n, n, n), dtype=np.int32)
    labels[n // 2:] = 1
    q = shoemake_quaternions(np.random.default_rng(5).random((2, 3)))
    laws = np.array([0, lawB], dtype=np.int32)
    rve = rve_from_labels(n, labels.ravel(), q, laws, op)
    hist = [(macro_F(e), 0.1) for e in (0.002, 0.004, 0.002)]
    ref = _laminate_reference(q, 0, lawB, hist, 0.5)
    for (Fb, dt), (FA, FB) in zip(hist, ref):
        info = rve.increment(Fb, dt, **TIGHT)
        assert info.status == OK
        F = rve.F.reshape(n, n, n, 3, 3)
        assert np.max(np.abs(F[:n // 2] - FA)) < 1e-10
        assert np.max(np.abs(F[n // 2:] - FB)) < 1e-10


def _dense_newton(rve, Pr, Fb_new, dt, tol=1e-12):
    """Newton with dense least-squares steps on the range of G."""
    N = rve.N
    F = rve.F + (Fb_new - rve.F_bar)[None]

    def vec(A):
        return A.reshape(N, 9).T.reshape(-1)

    def unvec(x):
        return x.reshape(9, N).T.reshape(N, 3, 3)

    dg = np.zeros((N, 12))
    for _ in range(40):
        Pf, K, trial, fails = rve.constitutive(F, dt, dg)
        assert fails == 0
        r = Pr @ vec(Pf)
        if np.linalg.norm(r) <= tol * np.linalg.norm(Pf):
            return F
        Kb = np.zeros((9 * N, 9 * N))
        Kv = K.reshape(N, 9, 9)
        for a in range(9):
            for b in range(9):
                Kb[a * N + np.arange(N), b * N + np.arange(N)] = Kv[:, a, b]
        A = Pr @ Kb @ Pr
        y = np.linalg.lstsq(A, -r, rcond=1e-12)[0]
        F = F + unvec(Pr @ y)
        dg = trial["dg"]
    raise AssertionError("dense Newton did not converge")


@pytest.mark.parametrize("n,op,indep", [(4, "continuous", False),
                                        (4, "discrete", False),
                                        (5, "continuous", True)])
def test_dense_brute_force_newton(n, op, indep):
    rng = np.random.default_rng(n)
    labels = rng.integers(0, 3, size=n ** 3).astype(np.int32)
    q = shoemake_quaternions(rng.random((3, 3)))
    rve = rve_from_labels(n, labels, q, operator=op)
    ref = rve_from_labels(n, labels, q, operator=op)
    if indep:
        D = fourier_diff_matrix(n, 1.0)
        Pr = range_projector(gradient_matrix(D, D, D))
    else:
        Pr = dense_G((n, n, n), (1, 1, 1), op)
    for eps in (0.002, 0.004):
        Fd = _dense_newton(ref, Pr, macro_F(eps), 0.1)
        info = rve.increment(macro_F(eps), 0.1, **TIGHT)
        assert info.status == OK
        assert np.max(np.abs(rve.F - Fd)) < 1e-10
        # advance the reference with the converged field and the same law
        ref.increment(macro_F(eps), 0.1, **TIGHT)


def _small_rve(n=8, G=4, seed=3, op="discrete"):
    rng = np.random.default_rng(seed)
    from synthetic.micro import voronoi_periodic
    labels = voronoi_periodic(n, rng.random((G, 3)))
    q = shoemake_quaternions(rng.random((G, 3)))
    return rve_from_labels(n, labels, q, operator=op)


def test_newton_jacobian_directional_fd():
    rve = _small_rve()
    rve.increment(macro_F(0.003), 0.1, **TIGHT)
    F = rve.F + (macro_F(0.004) - rve.F_bar)[None]
    dg0 = np.zeros((rve.N, 12))
    _, K, _, _ = rve.constitutive(F, 0.1, dg0)
    v = rve.G(RNG.standard_normal((rve.N, 3, 3))) * 1e-3
    h = 1e-5
    Pp = rve.constitutive(F + h * v, 0.1, dg0)[0]
    Pm = rve.constitutive(F - h * v, 0.1, dg0)[0]
    fd = rve.G((Pp - Pm) / (2 * h))
    an = rve.G(np.einsum("vijkl,vkl->vij", K, v))
    assert np.max(np.abs(fd - an)) < 1e-6 * np.max(np.abs(an))


def test_mean_hill_mandel_and_quadratic_rate():
    rve = _small_rve(op="continuous")
    for eps in (0.002, 0.004):
        info = rve.increment(macro_F(eps), 0.1, **TIGHT)
        assert info.status == OK
        assert np.max(np.abs(rve.F.mean(axis=0) - macro_F(eps))) < 1e-14
        Ft = rve.F - macro_F(eps)
        hm = np.mean(np.einsum("vij,vij->v", rve.P, Ft))
        scale = np.mean(np.linalg.norm(rve.P.reshape(-1, 9), axis=1)
                        * np.linalg.norm(Ft.reshape(-1, 9), axis=1))
        assert abs(hm) < 1e-10 * scale
        res = [r for r in info.residuals if r > 1e-13]
        # quadratic: the exponent of the last useful reduction approaches 2
        assert len(res) >= 3
        rates = [np.log(res[i + 1]) / np.log(res[i])
                 for i in range(len(res) - 1) if res[i] < 1e-2]
        assert rates and max(rates) > 1.7


def test_failed_increment_rolls_back():
    rve = _small_rve()
    rve.increment(macro_F(0.002), 0.1)
    snap = {k: getattr(rve, k).copy() for k in ("F", "Fpi", "chi", "pcyc",
                                                "wcyc", "P")}
    info = rve.increment(macro_F(0.03), 0.1, newton_max=1)
    assert info.status == ENOTCONV
    for k, v in snap.items():
        assert np.array_equal(getattr(rve, k), v)
    rve.F[5, 0, 0] = np.nan
    info = rve.increment(macro_F(0.003), 0.1)
    assert info.status == ELOCAL and info.local_failures >= 1
    assert np.array_equal(rve.Fpi, snap["Fpi"])
