"""Pins of the oracle's constitutive laws (CPU only).

* tangents against central finite differences of P(F) (brute force);
* the elastic limit against the closed-form St-Venant-Kirchhoff stress;
* objectivity P(QF) = Q P(F) and invariance under the cubic symmetry group;
* the single crystal in the lattice frame under the uniaxial macro gradient
  of Eq. 27: eight equivalent systems reduce the law to one scalar
  backward-Euler equation, solved here independently by bisection.
"""

import numpy as np
import pytest

from oracle import crystal, material
from synthetic import material_params, shoemake_quaternions, macro_F

P = material_params()
RNG = np.random.default_rng(7)


def _grains(M, seed=0):
    q = shoemake_quaternions(np.random.default_rng(seed).random((M, 3)))
    return crystal.grain_tables(q, P)


def test_slip_systems_geometry():
    s, m = crystal.fcc_slip_systems()
    assert s.shape == (12, 3)
    assert np.allclose(np.linalg.norm(s, axis=1), 1)
    assert np.allclose(np.linalg.norm(m, axis=1), 1)
    assert np.allclose(np.sum(s * m, axis=1), 0)
    S0 = np.einsum("ai,aj->aij", s, m).reshape(12, 9)
    # 12 distinct systems; Schmid tensors span the 5-dim deviatoric space
    # plus spins, and are traceless
    assert np.linalg.matrix_rank(S0) == 8
    assert np.allclose(np.einsum("aii->a", S0.reshape(12, 3, 3)), 0)


def test_quaternion_matrix():
    assert np.allclose(crystal.quat_to_matrix([1, 0, 0, 0]), np.eye(3))
    c = np.cos(np.pi / 4)
    Rz = crystal.quat_to_matrix([c, 0, 0, c])          # +90 deg about z
    assert np.allclose(Rz @ [1, 0, 0], [0, 1, 0])
    for q in shoemake_quaternions(RNG.random((20, 3))):
        R = crystal.quat_to_matrix(q)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14


def test_cubic_stiffness_uniaxial_and_symmetries():
    C = crystal.cubic_stiffness(P[0], P[1], P[2])
    assert C[0, 0, 0, 0] == P[0] and C[0, 0, 1, 1] == P[1]
    assert C[0, 1, 0, 1] == P[2]
    R = crystal.quat_to_matrix(shoemake_quaternions(RNG.random((1, 3)))[0])
    Cr = crystal.rotate4(C, R)
    for perm in ("jikl", "ijlk", "klij"):
        assert np.allclose(Cr, np.einsum("ijkl->" + perm, Cr))
    # rotation invariants: bulk part and the Frobenius norm
    assert np.isclose(np.einsum("iijj", Cr), np.einsum("iijj", C))
    assert np.isclose(np.sum(Cr * Cr), np.sum(C * C))


def _fd_tangent(fun, F, h=1e-7):
    K = np.zeros(F.shape[:1] + (3, 3, 3, 3))
    for k in range(3):
        for l in range(3):
            Fp, Fm = F.copy(), F.copy()
            Fp[:, k, l] += h
            Fm[:, k, l] -= h
            K[:, :, :, k, l] = (fun(Fp) - fun(Fm)) / (2 * h)
    return K


@pytest.mark.parametrize("amp,chi_amp", [(6e-4, 0.0), (3e-3, 40.0),
                                         (1e-2, 90.0)])
def test_cp_tangent_matches_finite_differences(amp, chi_amp):
    M = 6
    S0, C = _grains(M, seed=int(amp * 1e4))
    F = np.eye(3) + amp * RNG.standard_normal((M, 3, 3))
    Fpi0 = np.eye(3) + 1e-3 * RNG.standard_normal((M, 3, 3))
    chi0 = chi_amp * np.tanh(RNG.standard_normal((M, 12)))
    dt = 0.1
    out = material.cp_update(F, Fpi0, chi0, np.zeros((M, 12)), S0, C, P, dt)
    assert out["ok"].all()

    def fun(Fx):
        return material.cp_update(Fx, Fpi0, chi0, out["dg"], S0, C, P, dt,
                                  tangent=False)["P"]

    K = _fd_tangent(fun, F)
    err = np.max(np.abs(K - out["K"])) / np.max(np.abs(K))
    assert err < 1e-6


def test_svk_tangent_matches_finite_differences():
    lam, mu = crystal.lame_from_young(P[8], P[9])
    assert np.isclose(lam, 480000.0) and np.isclose(mu, 480000.0)
    F = np.eye(3) + 5e-3 * RNG.standard_normal((5, 3, 3))
    out = material.svk_update(F, lam, mu)
    K = _fd_tangent(lambda Fx: material.svk_update(Fx, lam, mu, False)["P"], F)
    assert np.max(np.abs(K - out["K"])) / np.max(np.abs(K)) < 1e-7


def test_elastic_limit_is_anisotropic_svk():
    # |tau - chi| << g: slips are ~ dt gdot0 (tau/g)^20, negligible
    M = 4
    S0, C = _grains(M, seed=3)
    F = np.eye(3) + 2e-5 * RNG.standard_normal((M, 3, 3))
    I = np.broadcast_to(np.eye(3), (M, 3, 3)).copy()
    out = material.cp_update(F, I, np.zeros((M, 12)), np.zeros((M, 12)),
                             S0, C, P, 0.1)
    E = 0.5 * (np.swapaxes(F, 1, 2) @ F - np.eye(3))
    S = np.einsum("mijkl,mkl->mij", C, E)
    P_ref = F @ S
    assert np.max(np.abs(out["P"] - P_ref)) < 1e-10 * np.max(np.abs(P_ref))


def test_objectivity_and_cubic_symmetry():
    M = 3
    q = shoemake_quaternions(RNG.random((M, 3)))
    S0, C = crystal.grain_tables(q, P)
    F = np.eye(3) + 4e-3 * RNG.standard_normal((M, 3, 3))
    I = np.broadcast_to(np.eye(3), (M, 3, 3)).copy()
    z = np.zeros((M, 12))
    base = material.cp_update(F, I, z, z, S0, C, P, 0.1)
    Q = crystal.quat_to_matrix(shoemake_quaternions(RNG.random((1, 3)))[0])
    rot = material.cp_update(Q @ F, I, z, z, S0, C, P, 0.1)
    assert np.max(np.abs(rot["P"] - Q @ base["P"])) < 1e-10 * np.max(
        np.abs(base["P"]))
    # lattice symmetry: orientation R and R H (H = 90 deg about lattice z)
    # describe the same crystal
    c = np.cos(np.pi / 4)
    H = np.array([c, 0.0, 0.0, c])
    qH = np.array([_qmul(qq, H) for qq in q])
    S0h, Ch = crystal.grain_tables(qH, P)
    sym = material.cp_update(F, I, z, z, S0h, Ch, P, 0.1)
    assert np.max(np.abs(sym["P"] - base["P"])) < 1e-9 * np.max(
        np.abs(base["P"]))
    assert np.allclose(np.sort(np.abs(sym["dg"]), axis=1),
                       np.sort(np.abs(base["dg"]), axis=1), rtol=1e-7,
                       atol=1e-15)


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


# ------------------------------------------- single crystal, scalar reduction
def scalar_single_crystal_step(f, p1_0, p2_0, chi0, dt, prm):
    """One backward-Euler step of the [100]-loaded crystal, by bisection.

    Eight systems carry |s1 m1| = 1/sqrt(6); their signed sum of Schmid
    tensors is diag(8, -4, -4)/sqrt(6).  Unknown: the common slip magnitude
    dgam (signed along that sum).  Returns dgam, chi, P1, P2, p1, p2, tau.
    """
    C11, C12 = prm[0], prm[1]
    gd0, g, n, c, d = prm[3], prm[4], prm[5], prm[6], prm[7]
    r6 = np.sqrt(6.0)

    def state(dgam):
        p1 = p1_0 * (1 - 8 * dgam / r6)
        p2 = p2_0 * (1 + 4 * dgam / r6)
        fe1, fe2 = f * p1, f ** -0.5 * p2
        E1, E2 = 0.5 * (fe1 * fe1 - 1), 0.5 * (fe2 * fe2 - 1)
        S1 = C11 * E1 + 2 * C12 * E2
        S2 = C12 * E1 + (C11 + C12) * E2
        tau = (S1 - S2) / r6
        chi = (chi0 + c * dgam) / (1 + d * abs(dgam))
        x = (tau - chi) / g
        R = dgam - dt * gd0 * abs(x) ** n * np.sign(x)
        return R, dict(chi=chi, P1=fe1 * S1 * p1, P2=fe2 * S2 * p2, p1=p1,
                       p2=p2, tau=tau)

    lo, hi = -0.05, 0.05
    assert state(lo)[0] < 0 < state(hi)[0]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if state(mid)[0] < 0:
            lo = mid
        else:
            hi = mid
    dgam = 0.5 * (lo + hi)
    return dgam, state(dgam)[1]


def test_single_crystal_schmid_reduces_to_scalar_law():
    S0, C = crystal.grain_tables(np.array([[1.0, 0, 0, 0]]), P)
    s, m = crystal.fcc_slip_systems()
    sgn = np.sign(np.round(np.sqrt(6) * s[:, 0] * m[:, 0], 12))
    active = sgn != 0
    assert active.sum() == 8
    Dsum = np.einsum("a,aij->ij", sgn, S0[0])
    assert np.allclose(Dsum, np.diag([8, -4, -4]) / np.sqrt(6), atol=1e-14)
    Fpi = np.eye(3)[None].copy()
    chi = np.zeros((1, 12))
    p1, p2, chis = 1.0, 1.0, 0.0
    dt = 0.1
    for eps in (0.002, 0.004, 0.006, 0.004, 0.0, -0.004, -0.006):
        F = macro_F(eps)
        out = material.cp_update(F[None], Fpi, chi, np.zeros((1, 12)), S0, C,
                                 P, dt)
        dgam, st = scalar_single_crystal_step(1 + eps, p1, p2, chis, dt, P)
        assert np.allclose(out["dg"][0, active], sgn[active] * dgam,
                           rtol=1e-9, atol=1e-16)
        assert np.allclose(out["dg"][0, ~active], 0.0, atol=1e-16)
        assert np.isclose(out["P"][0, 0, 0], st["P1"], rtol=1e-10)
        assert np.isclose(out["P"][0, 1, 1], st["P2"], rtol=1e-10)
        assert np.isclose(out["chi"][0, active][0] * sgn[active][0],
                          st["chi"], rtol=1e-9, atol=1e-10)
        Fpi, chi = out["Fpi"], out["chi"]
        p1, p2, chis = st["p1"], st["p2"], st["chi"]
    # the saturated back stress approaches c/d
    assert abs(chis) < P[6] / P[7] + 1e-9
