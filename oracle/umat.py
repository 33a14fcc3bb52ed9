"""Bridge from a finite-strain user material in the form of a commercial FE
code (Cauchy stress and the tangent of the Jaumann rate of the Kirchhoff
stress) to the quantities the FFT solver needs (oracle; test
infrastructure).

Appendix A of the paper:
  Eq. A.1   P = J sigma F^-T,   J = det F
  Eq. A.2   the user tangent C^ab: Jaumann rate of tau = J C^ab : d
  Eq. A.16  K_ijkl = ( J C^ab_ipkm F^-1_lm
                       + 1/2 d_ik F^-1_lm tau_mp - 1/2 F^-1_li tau_kp
                       + 1/2 d_pk F^-1_lm tau_im - 1/2 F^-1_lp tau_ik ) F^-1_jp
                     - tau_ip F^-1_lp F^-1_jk
with tau = J sigma.  The 6x6 tangent of such a material uses the component
order 11, 22, 33, 12, 13, 23 and engineering shear strains, so the tensor
C_ijkl is the matrix entry of the pair (ij, kl) for every index order.

``neo_hooke_umat`` is a user material in that form (the example material of
the user-material interface): a compressible neo-Hookean solid with per-voxel
moduli held in its state variables, and one history variable that sums
|J - J_prev| over converged increments (it has no effect on the stress; it
shows the commit semantics of state variables).

Pins: K against central finite differences of P(F) for the compressible
neo-Hookean material; P against its definition and against the textbook
neo-Hookean Piola stress; the Voigt convention against a strain-stress
product.  Status: pinned.
"""

from __future__ import annotations

import numpy as np

# component order of the 6x6 tangent: 11, 22, 33, 12, 13, 23
VOIGT_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def voigt_index():
    """v[i, j] = position of the pair (i, j) in the 6-vector."""
    v = np.zeros((3, 3), dtype=np.int64)
    for a, (i, j) in enumerate(VOIGT_PAIRS):
        v[i, j] = v[j, i] = a
    return v


def tensor_from_voigt(D):
    """(..., 6, 6) -> (..., 3, 3, 3, 3) with C_ijkl = D[v(ij), v(kl)]."""
    v = voigt_index()
    return np.asarray(D)[..., v[:, :, None, None], v[None, None, :, :]]


def sym_from_voigt(s):
    """(..., 6) stress in the order above -> (..., 3, 3)."""
    v = voigt_index()
    return np.asarray(s)[..., v]


def piola_from_cauchy(F, sigma):
    """Eq. A.1: P = J sigma F^-T (F, sigma: (..., 3, 3))."""
    J = np.linalg.det(F)
    Finv = np.linalg.inv(F)
    return J[..., None, None] * sigma @ np.swapaxes(Finv, -1, -2)


def tangent_from_jaumann(F, sigma, Cab):
    """Eq. A.16 (F, sigma: (..., 3, 3); Cab: (..., 3, 3, 3, 3))."""
    J = np.linalg.det(F)
    Fi = np.linalg.inv(F)              # Fi[a, b] = F^-1_ab
    tau = J[..., None, None] * sigma
    d = np.eye(3)
    # dtau_ip / dF_kl
    dtau = (J[..., None, None, None, None] * np.einsum("...ipkm,...lm->...ipkl", Cab, Fi)
            + 0.5 * np.einsum("ik,...lm,...mp->...ipkl", d, Fi, tau)
            - 0.5 * np.einsum("...li,...kp->...ipkl", Fi, tau)
            + 0.5 * np.einsum("pk,...lm,...im->...ipkl", d, Fi, tau)
            - 0.5 * np.einsum("...lp,...ik->...ipkl", Fi, tau))
    return (np.einsum("...ipkl,...jp->...ijkl", dtau, Fi)
            - np.einsum("...ip,...lp,...jk->...ijkl", tau, Fi, Fi))


def neo_hooke_umat(F1, F0, statev, dt):
    """Compressible neo-Hookean user material (F1, F0: (N, 3, 3); statev:
    (N, >=3) with mu, lambda, accumulated |dJ|).

    Kirchhoff stress tau = mu (B - I) + lambda ln J I with B = F1 F1^T; the
    Jaumann tangent J C^ab_ijkl = lambda d_ij d_kl + (mu - lambda ln J)
    (d_ik d_jl + d_il d_jk) + 1/2 (d_ik tau_jl + d_il tau_jk + tau_ik d_jl
    + tau_il d_jk).  Returns (sigma (N, 6), ddsdde (N, 6, 6), statev_new,
    ok (N,)), sigma and ddsdde in the 6-component order above.
    """
    F1 = np.asarray(F1, dtype=np.float64)
    mu = statev[:, 0][:, None, None]
    lam = statev[:, 1][:, None, None]
    J = np.linalg.det(F1)
    ok = np.isfinite(J) & (J > 0.0)
    Jc = np.where(ok, J, 1.0)
    lnJ = np.log(Jc)[:, None, None]
    I = np.eye(3)
    B = F1 @ np.swapaxes(F1, 1, 2)
    tau = mu * (B - I) + lam * lnJ * I
    c = (lam[..., None, None] * np.einsum("ij,kl->ijkl", I, I)
         + (mu - lam * lnJ)[..., None, None]
         * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)))
    extra = 0.5 * (np.einsum("ik,vjl->vijkl", I, tau)
                   + np.einsum("il,vjk->vijkl", I, tau)
                   + np.einsum("vik,jl->vijkl", tau, I)
                   + np.einsum("vil,jk->vijkl", tau, I))
    Cab = (c + extra) / Jc[:, None, None, None, None]
    sigma = tau / Jc[:, None, None]
    a = [p[0] for p in VOIGT_PAIRS]
    b = [p[1] for p in VOIGT_PAIRS]
    s6 = sigma[:, a, b]
    D = Cab[:, a, b][:, :, a, b]
    sv = np.array(statev, dtype=np.float64, copy=True)
    sv[:, 2] += np.abs(J - np.linalg.det(F0))
    return s6, D, sv, ok
