"""Projection operators and the linear map G (oracle).

* Fourier frequencies: Sec. 2.2, Eq. 18.
* Continuous operator Ghat: Sec. 2.2, Eq. 19.
* Discrete operator Ghat' (rotated centred differences): Sec. 2.2, Eqs. 20-21.
* G(A) = F^{-1}{ Ghat : F(A) }: Sec. 2.1, Eqs. 10-11.

Readings (listed in the design notes):
* The scaling printed in Eqs. 19 and 21 is not a valid index expression; the
  operator is taken as delta_ik v_j v_l / |v|^2 with the physical wave vector
  v_d = q_d n_d / L_d (continuous) or v_d = tan(q_d / 2) n_d / L_d (discrete).
  On a cubic grid of a cubic cell the scale cancels.
* "Null and Nyquist frequencies" are zeroed: k = 0, and every frequency with
  at least one component equal to -n_d/2 (only on even n_d).  This mask is
  applied to both operators.
* (Ghat : A)_ij = Ghat_ijkl A_kl (Notation table), which with the delta_ik
  structure is B_ij = v_j (sum_l A_il v_l) / |v|^2.

Pins: idempotence, self-adjointness, real output, zero mean, exact recovery
of compatible fields, annihilation of divergence-free rows, agreement of the
tan form with the complex form of Eq. 20, and the brute-force projector onto
the range of the real-space rotated-difference gradient.  Status: pinned.
"""

from __future__ import annotations

import numpy as np

from .dft import dft3, idft3_real

CONTINUOUS = "continuous"
DISCRETE = "discrete"


def paper_frequencies(n: int) -> np.ndarray:
    """Eq. 18: q^(i) for i = 1..n, in the paper's (descending) order."""
    i = np.arange(1, n + 1)
    if n % 2 == 0:
        return 2 * np.pi * (n / 2 - i) / n
    return 2 * np.pi * ((n + 1) / 2 - i) / n


def frequencies_dft_order(n: int):
    """Frequencies of Eq. 18 arranged by DFT index, plus the Nyquist mask.

    The integer frequency of q^(i) is k = q n / (2 pi); its DFT index is
    k mod n.  Returns (q, is_nyquist), both of length n, in DFT index order.
    """
    q_list = paper_frequencies(n)
    k_list = np.rint(q_list * n / (2 * np.pi)).astype(int)
    q = np.empty(n)
    nyq = np.zeros(n, dtype=bool)
    for qq, kk in zip(q_list, k_list):
        q[kk % n] = qq
        if n % 2 == 0 and kk == -n // 2:
            nyq[kk % n] = True
    return q, nyq


def wave_vectors(shape, L=(1.0, 1.0, 1.0), operator: str = CONTINUOUS):
    """Per-axis wave-vector components and the zero mask.

    Returns (v1, v2, v3, zero) where v_d has shape broadcastable over the
    (n1, n2, n3) frequency grid and ``zero`` marks the null frequency and
    every frequency with a Nyquist component.
    """
    vs = []
    nyqs = []
    for d, n in enumerate(shape):
        q, nyq = frequencies_dft_order(n)
        scale = n / L[d]
        if operator == CONTINUOUS:
            v = q * scale
        elif operator == DISCRETE:
            qs = np.where(nyq, 0.0, q)          # tan(pi/2) is never formed
            v = np.tan(qs / 2) * scale
        else:
            raise ValueError(f"unknown operator {operator!r}")
        sh = [1, 1, 1]
        sh[d] = n
        vs.append(v.reshape(sh))
        nyqs.append(nyq.reshape(sh))
    zero = (nyqs[0] | nyqs[1] | nyqs[2])
    zero = np.broadcast_to(zero, tuple(shape)).copy()
    zero[0, 0, 0] = True
    return vs[0], vs[1], vs[2], zero


def project_spectrum(Ahat: np.ndarray, L=(1.0, 1.0, 1.0),
                     operator: str = CONTINUOUS) -> np.ndarray:
    """Bhat_ij = v_j sum_l Ahat_il v_l / |v|^2, zero on the masked set.

    ``Ahat`` has shape (3, 3, n1, n2, n3) (complex).
    """
    shape = Ahat.shape[2:]
    v1, v2, v3, zero = wave_vectors(shape, L, operator)
    v = [np.broadcast_to(x, shape) for x in (v1, v2, v3)]
    nrm2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    inv = np.where(zero, 0.0, 1.0 / np.where(zero, 1.0, nrm2))
    B = np.zeros_like(Ahat, dtype=np.complex128)
    for i in range(3):
        s = Ahat[i, 0] * v[0] + Ahat[i, 1] * v[1] + Ahat[i, 2] * v[2]
        s = s * inv
        for j in range(3):
            B[i, j] = v[j] * s
    return B


def apply_G(A: np.ndarray, L=(1.0, 1.0, 1.0),
            operator: str = CONTINUOUS) -> np.ndarray:
    """Eq. 11: G(A) = F^{-1}{Ghat : F(A)} for a real field (3, 3, n1, n2, n3)."""
    A = np.asarray(A, dtype=np.float64)
    scale = float(np.max(np.abs(A))) if A.size else 0.0
    return idft3_real(project_spectrum(dft3(A), L, operator), scale=scale)


def apply_G_complex_willot(A: np.ndarray, L=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Discrete operator from the complex modified wave vector of Eq. 20.

    q'_d = (1/4) tan(q_d/2) prod_m (1 + exp(i q_m)), each scaled by n_d/L_d,
    and Ghat'_ijkl = delta_ik q'_j conj(q'_l) / |q'|^2 on the non-masked set.
    Used to check that the real tan form of Eq. 21 follows from Eq. 20.
    """
    A = np.asarray(A, dtype=np.float64)
    Ahat = dft3(A)
    shape = A.shape[2:]
    qs, nyqs = [], []
    for d, n in enumerate(shape):
        q, nyq = frequencies_dft_order(n)
        sh = [1, 1, 1]
        sh[d] = n
        qs.append(np.broadcast_to(q.reshape(sh), shape))
        nyqs.append(np.broadcast_to(nyq.reshape(sh), shape))
    zero = nyqs[0] | nyqs[1] | nyqs[2]
    zero = zero.copy()
    zero[0, 0, 0] = True
    common = (1 + np.exp(1j * qs[0])) * (1 + np.exp(1j * qs[1])) * \
             (1 + np.exp(1j * qs[2]))
    kv = []
    for d in range(3):
        qd = np.where(zero, 0.0, qs[d])
        kv.append(0.25 * np.tan(qd / 2) * common * (shape[d] / L[d]))
    nrm2 = sum(np.abs(k) ** 2 for k in kv)
    inv = np.where(zero, 0.0, 1.0 / np.where(zero | (nrm2 == 0), 1.0, nrm2))
    B = np.zeros_like(Ahat)
    for i in range(3):
        s = sum(Ahat[i, l] * np.conj(kv[l]) for l in range(3)) * inv
        for j in range(3):
            B[i, j] = kv[j] * s
    return idft3_real(B, scale=float(np.max(np.abs(A))))


def dense_G(shape, L=(1.0, 1.0, 1.0), operator: str = CONTINUOUS) -> np.ndarray:
    """The (9N x 9N) matrix of the linear map G, column by column (tiny grids).

    Row/column index = c * N + v with c = 3 i + j and v the flat voxel index.
    """
    N = int(np.prod(shape))
    M = np.zeros((9 * N, 9 * N))
    e = np.zeros((9 * N,))
    for col in range(9 * N):
        e[:] = 0.0
        e[col] = 1.0
        M[:, col] = apply_G(e.reshape((3, 3) + tuple(shape)), L,
                            operator).reshape(-1)
    return M
