"""Pins of the Appendix A bridge (oracle/umat.py): Eq. A.1 and Eq. A.16
against finite differences of P(F) for a compressible neo-Hookean material
whose Cauchy stress and Jaumann tangent are known in closed form."""

import numpy as np
import pytest

from oracle import umat

MU, LAM = 80.0, 120.0


def neo_hooke(F):
    """Kirchhoff stress tau = mu (B - I) + lam ln J I, its Cauchy stress and
    the tangent of the Jaumann rate, J C^ab = c + (d tau + tau d) terms with
    c = lam I (x) I + 2 (mu - lam ln J) I_sym."""
    J = np.linalg.det(F)
    B = F @ F.T
    I = np.eye(3)
    tau = MU * (B - I) + LAM * np.log(J) * I
    c = (LAM * np.einsum("ij,kl->ijkl", I, I)
         + (MU - LAM * np.log(J)) * (np.einsum("ik,jl->ijkl", I, I)
                                      + np.einsum("il,jk->ijkl", I, I)))
    extra = 0.5 * (np.einsum("ik,lj->ijkl", I, tau) + np.einsum("il,kj->ijkl", I, tau)
                   + np.einsum("ik,jl->ijkl", tau, I) + np.einsum("il,jk->ijkl", tau, I))
    return tau / J, (c + extra) / J


def piola(F):
    sigma, _ = neo_hooke(F)
    return umat.piola_from_cauchy(F, sigma)


def random_F(rng, amp=0.2):
    F = np.eye(3) + amp * rng.standard_normal((3, 3))
    if np.linalg.det(F) <= 0.2:
        F = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
    return F


def test_piola_from_cauchy_definition():
    rng = np.random.default_rng(0)
    F = random_F(rng)
    s = rng.standard_normal((3, 3))
    s = s + s.T
    P = umat.piola_from_cauchy(F, s)
    # P F^T = J sigma
    assert np.allclose(P @ F.T, np.linalg.det(F) * s, rtol=1e-13, atol=1e-13)


def test_voigt_convention_engineering_shear():
    rng = np.random.default_rng(1)
    D = rng.standard_normal((6, 6))
    C = umat.tensor_from_voigt(D)
    e = rng.standard_normal((3, 3))
    e = 0.5 * (e + e.T)
    ev = np.array([e[0, 0], e[1, 1], e[2, 2], 2 * e[0, 1], 2 * e[0, 2], 2 * e[1, 2]])
    ds = D @ ev
    dS = np.einsum("ijkl,kl->ij", C, e)
    v = umat.voigt_index()
    assert np.allclose(dS[[0, 1, 2, 0, 0, 1], [0, 1, 2, 1, 2, 2]], ds, rtol=1e-13)
    assert np.allclose(umat.sym_from_voigt(np.arange(6.0))[v == 3], 3.0)


def test_tangent_matches_finite_differences_of_P():
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(5):
        F = random_F(rng)
        sigma, Cab = neo_hooke(F)
        K = umat.tangent_from_jaumann(F, sigma, Cab)
        Kfd = np.zeros((3, 3, 3, 3))
        for k in range(3):
            for l in range(3):
                E = np.zeros((3, 3))
                E[k, l] = h
                Kfd[:, :, k, l] = (piola(F + E) - piola(F - E)) / (2 * h)
        err = np.max(np.abs(K - Kfd)) / np.max(np.abs(Kfd))
        assert err < 1e-8, err


def test_tangent_at_identity_is_the_small_strain_tangent_plus_stress_terms():
    # at F = I with zero stress the bridge returns the user tangent itself
    I = np.eye(3)
    sigma, Cab = neo_hooke(I)
    assert np.allclose(sigma, 0.0)
    K = umat.tangent_from_jaumann(I, sigma, Cab)
    assert np.allclose(K, Cab, rtol=1e-14, atol=1e-12)


# ---------------------------------------------------------------------------
# the example user material and the increment algorithm driven through the
# bridge (oracle.solver.OracleUmatRVE)

from oracle.solver import OracleUmatRVE, OK  # noqa: E402

TIGHT = dict(tol=1e-12, eta=1e-12, newton_max=40, cg_max=5000)


def neo_hooke_piola(F, mu, lam):
    """Textbook compressible neo-Hookean Piola stress
    P = mu (F - F^-T) + lam ln J F^-T."""
    FiT = np.linalg.inv(F).T
    return mu * (F - FiT) + lam * np.log(np.linalg.det(F)) * FiT


def _umat_at(F, mu=MU, lam=LAM):
    sv = np.array([[mu, lam, 0.0]])
    s6, D, sv1, ok = umat.neo_hooke_umat(F[None], np.eye(3)[None], sv, 0.1)
    sig = umat.sym_from_voigt(s6[0])
    return sig, umat.tensor_from_voigt(D[0]), sv1[0], ok[0]


def test_neo_hooke_umat_piola_is_the_textbook_stress():
    rng = np.random.default_rng(10)
    for _ in range(5):
        F = random_F(rng)
        sig, _, _, ok = _umat_at(F)
        assert ok
        P = umat.piola_from_cauchy(F, sig)
        assert np.allclose(P, neo_hooke_piola(F, MU, LAM), rtol=1e-12,
                           atol=1e-12 * MU)


def test_neo_hooke_umat_tangent_through_the_bridge_is_dP_dF():
    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(5):
        F = random_F(rng)
        sig, C, _, _ = _umat_at(F)
        K = umat.tangent_from_jaumann(F, sig, C)
        Kfd = np.zeros((3, 3, 3, 3))
        for k in range(3):
            for l in range(3):
                E = np.zeros((3, 3))
                E[k, l] = h
                Kfd[:, :, k, l] = (neo_hooke_piola(F + E, MU, LAM)
                                   - neo_hooke_piola(F - E, MU, LAM)) / (2 * h)
        assert np.max(np.abs(K - Kfd)) < 1e-8 * np.max(np.abs(Kfd))


def test_neo_hooke_umat_state_variables():
    rng = np.random.default_rng(12)
    F1 = np.stack([random_F(rng) for _ in range(4)])
    F0 = np.stack([random_F(rng) for _ in range(4)])
    sv = np.array([[1.0, 2.0, 0.5, 7.0]] * 4)
    _, _, sv1, ok = umat.neo_hooke_umat(F1, F0, sv, 0.1)
    assert ok.all()
    assert np.array_equal(sv1[:, [0, 1, 3]], sv[:, [0, 1, 3]])
    assert np.allclose(sv1[:, 2], 0.5 + np.abs(np.linalg.det(F1)
                                               - np.linalg.det(F0)))
    F1[2] = np.diag([1.0, 1.0, -1.0])
    assert not umat.neo_hooke_umat(F1, F0, sv, 0.1)[3][2]


def _macro(rng, amp=0.04):
    return np.eye(3) + amp * rng.standard_normal((3, 3))


def test_umat_rve_homogeneous_one_evaluation():
    n = 4
    sv = np.tile([MU, LAM, 0.0], (n ** 3, 1))
    rve = OracleUmatRVE((n, n, n), umat.neo_hooke_umat, sv)
    rng = np.random.default_rng(13)
    J_prev = 1.0
    acc = 0.0
    for _ in range(3):
        Fb = _macro(rng)
        info = rve.increment(Fb, 0.1, **TIGHT)
        assert info.status == OK
        assert info.newton_iters == 0 and info.cg_iters_total == 0
        assert np.allclose(info.P_bar, neo_hooke_piola(Fb, MU, LAM),
                           rtol=1e-12, atol=1e-12 * MU)
        acc += abs(np.linalg.det(Fb) - J_prev)
        J_prev = np.linalg.det(Fb)
        assert np.allclose(rve.statev[:, 2], acc, rtol=1e-12)


def _laminate_neo_hooke(Fb, mA, mB, phiA=0.5):
    """Exact laminate: F_A = Fb + phiB c e1, F_B = Fb - phiA c e1 with
    continuous traction P e1, solved with the textbook stress."""
    phiB = 1.0 - phiA
    e1 = np.array([1.0, 0, 0])

    def r(c):
        FA = Fb + phiB * np.outer(c, e1)
        FB = Fb - phiA * np.outer(c, e1)
        return (neo_hooke_piola(FA, *mA) - neo_hooke_piola(FB, *mB))[:, 0]

    c = np.zeros(3)
    for _ in range(60):
        rc = r(c)
        if np.max(np.abs(rc)) < 1e-12 * mA[0]:
            break
        J = np.zeros((3, 3))
        for j in range(3):
            dc = np.zeros(3)
            dc[j] = 1e-7
            J[:, j] = (r(c + dc) - rc) / 1e-7
        c = c - np.linalg.solve(J, rc)
    return Fb + phiB * np.outer(c, e1), Fb - phiA * np.outer(c, e1)


@pytest.mark.parametrize("op", ["continuous", "discrete"])
def test_umat_rve_laminate_exact_solution(op):
    n = 8
    mA, mB = (MU, LAM), (6 * MU, 6 * LAM)
    sv = np.zeros((n, n, n, 3))
    sv[: n // 2] = [*mA, 0.0]
    sv[n // 2:] = [*mB, 0.0]
    rve = OracleUmatRVE((n, n, n), umat.neo_hooke_umat, sv.reshape(-1, 3), op)
    rng = np.random.default_rng(14)
    for _ in range(3):
        Fb = _macro(rng, 0.06)
        info = rve.increment(Fb, 0.1, **TIGHT)
        assert info.status == OK and info.newton_iters >= 2
        FA, FB = _laminate_neo_hooke(Fb, mA, mB)
        F = rve.F.reshape(n, n, n, 3, 3)
        assert np.max(np.abs(F[: n // 2] - FA)) < 1e-10
        assert np.max(np.abs(F[n // 2:] - FB)) < 1e-10


def test_umat_rve_newton_converges_quadratically():
    n = 6
    rng = np.random.default_rng(15)
    stiff = rng.random(n ** 3) < 0.3
    sv = np.where(stiff[:, None], [6 * MU, 6 * LAM, 0.0], [MU, LAM, 0.0])
    rve = OracleUmatRVE((n, n, n), umat.neo_hooke_umat, sv, "discrete")
    info = rve.increment(_macro(rng, 0.08), 0.1, **TIGHT)
    assert info.status == OK
    res = [r for r in info.residuals if r > 1e-13]
    assert len(res) >= 3
    # e_{k+1} <= C e_k^2 once in the quadratic regime
    for a, b in zip(res[1:-1], res[2:]):
        assert b < 10.0 * a * a or b < 1e-11
