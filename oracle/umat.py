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

Pins: K against central finite differences of P(F) for a compressible
neo-Hookean material whose Cauchy stress and Jaumann tangent are known in
closed form; P against its definition.  Status: pinned.
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
