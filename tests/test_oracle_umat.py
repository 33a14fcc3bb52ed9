"""Pins of the Appendix A bridge (oracle/umat.py): Eq. A.1 and Eq. A.16
against finite differences of P(F) for a compressible neo-Hookean material
whose Cauchy stress and Jaumann tangent are known in closed form."""

import numpy as np

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
