"""The CG step length of the GPU path (CPU only; pins a reading, not a kernel).

The CG of the text after Eq. 16 takes alpha = r.r / p.A p with
A p = G(K : p).  Every CG direction is a combination of outputs of G, and G
(Eqs. 19/21, zero at the null frequency and wherever a component is a
Nyquist frequency) is an orthogonal projection in the discrete inner
product, so p.G(K:p) = G(p).(K:p) = p.(K:p).  The GPU path forms alpha from
p.(K:p) in its direction kernel, before the FFT passes.  Checked here on the
oracle's own projection (itself pinned against the Fourier differentiation
matrix and the rotated-difference stencil), for both operators on an even
grid with Nyquist planes and a non-symmetric per-voxel tangent: the two dots
agree to rounding, and a CG run in that form reproduces the textbook CG.
"""

import numpy as np
import pytest

from oracle.projection import apply_G
from oracle.solver import cg

SHAPE = (6, 6, 6)


def _tangent(rng):
    # non-symmetric per-voxel 9x9 map, positive-definite symmetric part
    eye = np.eye(9).reshape(3, 3, 3, 3)
    noise = rng.standard_normal((3, 3, 3, 3) + SHAPE)
    return 3.0 * eye[..., None, None, None] + 0.4 * noise


def _apply_K(K, p):
    return np.einsum("ijklxyz,klxyz->ijxyz", K, p)


def _cg_kp_form(K, b, op, eta, maxit):
    """CG with alpha = r.r / p.(K:p) and r -= alpha G(K:p)."""
    x = np.zeros_like(b)
    r = b.copy()
    rr = float(np.vdot(r, r))
    bnorm = np.sqrt(rr)
    p = r.copy()
    it = 0
    while it < maxit:
        y = _apply_K(K, p)
        it += 1
        alpha = rr / float(np.vdot(p, y))
        x += alpha * p
        r -= alpha * apply_G(y, operator=op)
        rr_new = float(np.vdot(r, r))
        if np.sqrt(rr_new) <= eta * bnorm:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, it


@pytest.mark.parametrize("op", ["continuous", "discrete"])
def test_dot_with_projected_product_equals_plain_dot(op):
    rng = np.random.default_rng(20180627)
    K = _tangent(rng)
    for _ in range(3):
        p = apply_G(rng.standard_normal((3, 3) + SHAPE), operator=op)
        y = _apply_K(K, p)
        lhs = float(np.vdot(p, apply_G(y, operator=op)))
        rhs = float(np.vdot(p, y))
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(p) * np.linalg.norm(y)
    # a field outside the range of G: the identity must not hold (the check
    # above is not vacuous)
    q = rng.standard_normal((3, 3) + SHAPE)
    y = _apply_K(K, q)
    assert abs(float(np.vdot(q, apply_G(y, operator=op))) - float(np.vdot(q, y))) \
        > 1e-3 * np.linalg.norm(q) * np.linalg.norm(y)


@pytest.mark.parametrize("op", ["continuous", "discrete"])
def test_cg_in_kp_form_reproduces_textbook_cg(op):
    rng = np.random.default_rng(7)
    K = _tangent(rng)
    b = -apply_G(rng.standard_normal((3, 3) + SHAPE), operator=op)
    # the same twelve iterations of both forms (CG on a non-symmetric
    # tangent is not guaranteed to reach a tight tolerance; the iterates
    # are what must agree)
    x_ref, it_ref, bd = cg(lambda p: apply_G(_apply_K(K, p), operator=op), b,
                           0.0, 12)
    assert not bd and it_ref == 12
    x, it = _cg_kp_form(K, b, op, 0.0, 12)
    assert it == 12
    assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    # and they made progress
    r = b - apply_G(_apply_K(K, x), operator=op)
    assert np.linalg.norm(r) < 0.1 * np.linalg.norm(b)
