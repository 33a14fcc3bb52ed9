"""Crystal geometry and elasticity of the FCC grains (oracle).

Sec. 3.2: the grains deform plastically by glide on the 12 octahedral
{111}<110> systems.  The slip-system order, orientation convention and
elastic constants below are readings fixed for this implementation (the
paper's own tables belong to a law it only cites):

* Plane normals m, in order: (1,1,1), (-1,1,1), (1,-1,1), (1,1,-1), each
  normalised.  For each plane the directions s are taken, in order, from
  (1,-1,0), (1,0,-1), (0,1,-1), (1,1,0), (1,0,1), (0,1,1) (normalised),
  keeping those orthogonal to m.  Schmid tensor S0 = s (x) m.
* Orientation: unit quaternion (w, x, y, z) -> active rotation matrix R
  mapping lattice vectors to sample vectors.
* Cubic stiffness in the lattice frame:
  C_abcd = C12 d_ab d_cd + C44 (d_ac d_bd + d_ad d_bc)
           + (C11 - C12 - 2 C44) sum_e d_ae d_be d_ce d_de,
  rotated to the sample frame as R_ia R_jb R_kc R_ld C_abcd.

Pins: 12 distinct unit systems with s.m = 0; R orthogonal with det 1;
rotated stiffness keeps both symmetries and its invariants; the uniaxial
Schmid factors of the single-crystal test.  Status: pinned.
"""

from __future__ import annotations

import numpy as np

_NORMALS = np.array([[1, 1, 1], [-1, 1, 1], [1, -1, 1], [1, 1, -1]],
                    dtype=np.float64)
_DIRECTIONS = np.array([[1, -1, 0], [1, 0, -1], [0, 1, -1], [1, 1, 0],
                        [1, 0, 1], [0, 1, 1]], dtype=np.float64)


def fcc_slip_systems():
    """(s, m) arrays of shape (12, 3) in the lattice frame, unit vectors."""
    s_list, m_list = [], []
    for m in _NORMALS:
        for s in _DIRECTIONS:
            if abs(float(s @ m)) < 1e-12:
                s_list.append(s / np.linalg.norm(s))
                m_list.append(m / np.linalg.norm(m))
    s = np.array(s_list)
    m = np.array(m_list)
    assert s.shape == (12, 3)
    return s, m


def quat_to_matrix(q) -> np.ndarray:
    """Active rotation matrix of a unit quaternion (w, x, y, z)."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def cubic_stiffness(C11: float, C12: float, C44: float) -> np.ndarray:
    """Fourth-order cubic stiffness tensor (3,3,3,3) in the lattice frame."""
    d = np.eye(3)
    C = (C12 * np.einsum("ab,cd->abcd", d, d)
         + C44 * (np.einsum("ac,bd->abcd", d, d)
                  + np.einsum("ad,bc->abcd", d, d)))
    for e in range(3):
        C[e, e, e, e] += C11 - C12 - 2 * C44
    return C


def isotropic_stiffness(lam: float, mu: float) -> np.ndarray:
    d = np.eye(3)
    return (lam * np.einsum("ab,cd->abcd", d, d)
            + mu * (np.einsum("ac,bd->abcd", d, d)
                    + np.einsum("ad,bc->abcd", d, d)))


def rotate4(C: np.ndarray, R: np.ndarray) -> np.ndarray:
    return np.einsum("ia,jb,kc,ld,abcd->ijkl", R, R, R, R, C, optimize=True)


def grain_tables(quat: np.ndarray, params: np.ndarray):
    """Per-grain sample-frame Schmid tensors and stiffness.

    Returns S0 of shape (G, 12, 3, 3) and C of shape (G, 3, 3, 3, 3).
    """
    s_lat, m_lat = fcc_slip_systems()
    C_lat = cubic_stiffness(params[0], params[1], params[2])
    G = quat.shape[0]
    S0 = np.empty((G, 12, 3, 3))
    C = np.empty((G, 3, 3, 3, 3))
    for g in range(G):
        R = quat_to_matrix(quat[g])
        s = s_lat @ R.T
        m = m_lat @ R.T
        S0[g] = np.einsum("ai,aj->aij", s, m)
        C[g] = rotate4(C_lat, R)
    return S0, C


def lame_from_young(E: float, nu: float):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return lam, mu
