"""Pins of the oracle's DFT and projection operators (CPU only).

What fixes the answer here is mathematics the paper relies on, not the
oracle's own formulas:
* the DFT definition summed voxel by voxel, and a library FFT;
* the continuous operator of Eq. 19 is the orthogonal projector onto the
  gradients of trigonometric-polynomial displacements: checked against the
  textbook Fourier differentiation matrix (Trefethen, Spectral Methods in
  MATLAB, ch. 3) on odd grids, including anisotropic cells;
* the discrete operator of Eq. 21 is the orthogonal projector onto gradients
  computed by rotated centred differences of a corner displacement field
  (Sec. 2.2, text before Eq. 20): checked against that real-space stencil;
* Eq. 21 follows from the complex modified wave vector of Eq. 20;
* idempotence, self-adjointness, zero mean, exact recovery of compatible
  fields, annihilation of fields with rows orthogonal to the wave vector,
  the rank of the dense operator.
"""

import os

import numpy as np
import pytest

from oracle import dft
from oracle.projection import (apply_G, apply_G_complex_willot, dense_G,
                               frequencies_dft_order, paper_frequencies)

RNG = np.random.default_rng(12345)


# ----------------------------------------------------------------- DFT (P1)
def test_dft_matches_definition_voxel_by_voxel():
    shape = (3, 4, 5)
    A = RNG.standard_normal(shape)
    B = dft.dft3(A)
    ref = np.zeros(shape, dtype=complex)
    for k in np.ndindex(*shape):
        s = 0j
        for x in np.ndindex(*shape):
            s += A[x] * np.exp(-2j * np.pi * sum(
                k[d] * x[d] / shape[d] for d in range(3)))
        ref[k] = s
    assert np.max(np.abs(B - ref)) < 1e-12


def test_dft_round_trip_and_library_fft():
    A = RNG.standard_normal((2, 3, 6, 5, 8))
    B = dft.dft3(A)
    assert np.allclose(B, np.fft.fftn(A, axes=(-3, -2, -1)), atol=1e-11,
                       rtol=0)
    assert np.max(np.abs(dft.idft3(B).real - A)) < 1e-13


# ------------------------------------------------------------ Eq. 18 values
def test_paper_frequencies_even_and_odd():
    # Eq. 18, listed by hand for n = 4..8 (tests/golden/eq18_frequencies.txt)
    path = os.path.join(os.path.dirname(__file__), "golden",
                        "eq18_frequencies.txt")
    rows = [list(map(int, l.split())) for l in open(path)
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for n, *m in rows:
        assert len(m) == n
        assert np.allclose(paper_frequencies(n), 2 * np.pi * np.array(m) / n,
                           rtol=0, atol=1e-15)
    q, nyq = frequencies_dft_order(4)
    assert np.allclose(q, [0.0, np.pi / 2, -np.pi, -np.pi / 2])
    assert list(nyq) == [False, False, True, False]
    q, nyq = frequencies_dft_order(5)
    assert not nyq.any()


# ------------------------------------------- independent real-space projectors
def fourier_diff_matrix(n, L):
    """Textbook Fourier differentiation matrix on n (odd) periodic points."""
    assert n % 2 == 1
    D = np.zeros((n, n))
    h = 2 * np.pi / n
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = 0.5 * (-1) ** (i - j) / np.sin((i - j) * h / 2)
    return D * (2 * np.pi / L)


def gradient_matrix(D1, D2, D3):
    """(9N x 3N) gradient operator from per-axis derivative matrices.

    Row (i, j, v) -> (3 i + j) N + v; column (i, v) -> i N + v; C order.
    """
    n1, n2, n3 = D1.shape[0], D2.shape[0], D3.shape[0]
    I1, I2, I3 = np.eye(n1), np.eye(n2), np.eye(n3)
    Dj = [np.kron(np.kron(D1, I2), I3), np.kron(np.kron(I1, D2), I3),
          np.kron(np.kron(I1, I2), D3)]
    N = n1 * n2 * n3
    G = np.zeros((9 * N, 3 * N))
    for i in range(3):
        for j in range(3):
            G[(3 * i + j) * N:(3 * i + j + 1) * N, i * N:(i + 1) * N] = Dj[j]
    return G


def rotated_difference_gradient(shape, L):
    """(9N x 3N): d u_i / d x_j at voxel centres from corner displacements.

    Corner (a, b, c) sits at (a h1, b h2, c h3); voxel (a, b, c) has the
    corners (a + s1, b + s2, c + s3), s in {0, 1}.  The derivative along j is
    the average of the differences along the four voxel edges parallel to j.
    """
    n = shape
    h = [L[d] / n[d] for d in range(3)]
    N = n[0] * n[1] * n[2]

    def flat(a, b, c):
        return ((a % n[0]) * n[1] + (b % n[1])) * n[2] + (c % n[2])

    Dj = [np.zeros((N, N)) for _ in range(3)]
    for a in range(n[0]):
        for b in range(n[1]):
            for c in range(n[2]):
                v = flat(a, b, c)
                for s1 in (0, 1):
                    for s2 in (0, 1):
                        for s3 in (0, 1):
                            corner = flat(a + s1, b + s2, c + s3)
                            s = (s1, s2, s3)
                            for j in range(3):
                                sign = 1.0 if s[j] == 1 else -1.0
                                Dj[j][v, corner] += sign / (4 * h[j])
    G = np.zeros((9 * N, 3 * N))
    for i in range(3):
        for j in range(3):
            G[(3 * i + j) * N:(3 * i + j + 1) * N, i * N:(i + 1) * N] = Dj[j]
    return G


def range_projector(Dg):
    U, s, _ = np.linalg.svd(Dg, full_matrices=False)
    r = int(np.sum(s > 1e-10 * s[0]))
    return U[:, :r] @ U[:, :r].T


@pytest.mark.parametrize("shape,L", [((3, 3, 3), (1.0, 1.0, 1.0)),
                                     ((5, 3, 3), (1.0, 2.0, 0.5)),
                                     ((3, 5, 3), (0.7, 1.0, 1.3))])
def test_continuous_operator_is_projector_onto_spectral_gradients(shape, L):
    Dg = gradient_matrix(*(fourier_diff_matrix(shape[d], L[d])
                           for d in range(3)))
    ref = range_projector(Dg)
    M = dense_G(shape, L, "continuous")
    assert np.max(np.abs(M - ref)) < 1e-12


@pytest.mark.parametrize("shape,L", [((3, 3, 3), (1.0, 1.0, 1.0)),
                                     ((5, 3, 3), (1.0, 2.0, 0.5)),
                                     ((3, 3, 5), (2.0, 1.0, 1.0))])
def test_discrete_operator_is_projector_onto_rotated_differences(shape, L):
    ref = range_projector(rotated_difference_gradient(shape, L))
    M = dense_G(shape, L, "discrete")
    assert np.max(np.abs(M - ref)) < 1e-12


def test_discrete_recovers_band_limited_rotated_gradient_on_even_grid():
    # On even grids the paper zeroes the Nyquist frequencies; a corner field
    # without Nyquist content has a rotated-difference gradient without it.
    shape, L = (8, 6, 4), (1.0, 1.5, 0.75)
    u = RNG.standard_normal((3,) + shape)
    U = np.fft.fftn(u, axes=(1, 2, 3))
    for d, n in enumerate(shape):
        sl = [slice(None)] * 4
        sl[d + 1] = n // 2
        U[tuple(sl)] = 0.0
    u = np.fft.ifftn(U, axes=(1, 2, 3)).real
    Dg = rotated_difference_gradient(shape, L)
    grad = (Dg @ u.reshape(-1)).reshape((3, 3) + shape)
    out = apply_G(grad, L, "discrete")
    assert np.max(np.abs(out - grad)) < 1e-12 * np.max(np.abs(grad))


# -------------------------------------------------------- invariants (P2, P3)
@pytest.mark.parametrize("op", ["continuous", "discrete"])
@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 4, 4), (5, 5, 5)])
def test_dense_operator_symmetric_idempotent_rank(op, shape):
    M = dense_G(shape, (1.0, 1.0, 1.0), op)
    assert np.max(np.abs(M - M.T)) < 1e-14
    assert np.max(np.abs(M @ M - M)) < 1e-13
    expected = {(3, 3, 3): 78, (4, 4, 4): 78, (5, 5, 5): 372}[shape]
    assert np.linalg.matrix_rank(M, tol=1e-8) == expected


@pytest.mark.parametrize("op", ["continuous", "discrete"])
def test_random_field_zero_mean_real_and_idempotent(op):
    A = RNG.standard_normal((3, 3, 8, 6, 10))
    B = apply_G(A, (1.0, 1.0, 1.0), op)
    assert np.max(np.abs(B.mean(axis=(2, 3, 4)))) < 1e-14
    assert np.max(np.abs(apply_G(B, (1.0, 1.0, 1.0), op) - B)) < 1e-13


def test_continuous_recovers_analytic_gradient():
    # u_i(x) = a_i sin(2 pi k.x + phi) for a few non-Nyquist modes: its exact
    # gradient sampled at voxel centres is a trigonometric polynomial field.
    n = (8, 10, 6)
    L = (1.0, 2.0, 0.5)
    x = [(np.arange(n[d]) + 0.5) * L[d] / n[d] for d in range(3)]
    X = np.meshgrid(*x, indexing="ij")
    grad = np.zeros((3, 3) + n)
    for _ in range(4):
        k = [RNG.integers(-n[d] // 2 + 1, n[d] // 2) for d in range(3)]
        a = RNG.standard_normal(3)
        phi = RNG.random() * 2 * np.pi
        arg = sum(2 * np.pi * k[d] * X[d] / L[d] for d in range(3)) + phi
        for i in range(3):
            for j in range(3):
                grad[i, j] += a[i] * np.cos(arg) * 2 * np.pi * k[j] / L[j]
    out = apply_G(grad, L, "continuous")
    assert np.max(np.abs(out - grad)) < 1e-12 * np.max(np.abs(grad))


@pytest.mark.parametrize("op", ["continuous", "discrete"])
def test_rows_orthogonal_to_wave_vector_are_annihilated(op):
    # A_ij = a_i b_j cos(2 pi k.x) with b orthogonal to k (cubic cell) is
    # divergence free row by row; both operators map it to zero because the
    # discrete wave vector of a single-axis mode is parallel to k.
    n = 8
    x = (np.arange(n) + 0.5) / n
    X = np.meshgrid(x, x, x, indexing="ij")
    k = np.array([0, 3, 0])
    b = np.array([1.0, 0.0, -2.0])
    a = RNG.standard_normal(3)
    arg = 2 * np.pi * (k[1] * X[1])
    A = np.einsum("i,j,abc->ijabc", a, b, np.cos(arg))
    assert np.max(np.abs(apply_G(A, (1, 1, 1), op))) < 1e-13


def test_tan_form_equals_complex_willot_form():
    A = RNG.standard_normal((3, 3, 6, 5, 4))
    L = (1.0, 0.8, 1.3)
    d1 = apply_G(A, L, "discrete")
    d2 = apply_G_complex_willot(A, L)
    assert np.max(np.abs(d1 - d2)) < 1e-13


def test_operators_agree_on_single_axis_fields():
    # P4: when the field varies along one axis only, q_2 = q_3 = 0 and both
    # wave vectors point along that axis.
    n = 12
    A = np.zeros((3, 3, n, n, n))
    prof = RNG.standard_normal((3, 3, n))
    A[:] = prof[:, :, :, None, None]
    c = apply_G(A, (1, 1, 1), "continuous")
    d = apply_G(A, (1, 1, 1), "discrete")
    assert np.max(np.abs(c - d)) < 1e-14 * max(1.0, np.max(np.abs(A)))


def test_discrete_minus_continuous_vanishes_at_low_frequency():
    # P4 trend: Ghat' - Ghat = O(|q|^2) as the mode gets smoother.
    errs = []
    for n in (8, 16, 32):
        x = (np.arange(n) + 0.5) / n
        X = np.meshgrid(x, x, x, indexing="ij")
        arg = 2 * np.pi * (X[0] + 2 * X[1] + X[2])
        A = np.einsum("ij,abc->ijabc", np.arange(9.0).reshape(3, 3) + 1,
                      np.cos(arg))
        errs.append(np.max(np.abs(apply_G(A, (1, 1, 1), "continuous")
                                  - apply_G(A, (1, 1, 1), "discrete"))))
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3
