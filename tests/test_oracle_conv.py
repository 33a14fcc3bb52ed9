"""Pins of the oracle's warm-start network (CPU only).

* forward convolution against a voxel-by-voxel direct sum with explicit
  periodic wrap-around (brute force, tiny grid);
* circular padding: translating the input translates the output;
* backward (data, weight, bias) against central finite differences of the
  loss in FP64;
* Adam against its update written out for one scalar.
"""

import numpy as np
import pytest

from oracle import conv

RNG = np.random.default_rng(2024)


def test_forward_matches_direct_sum():
    n, ci, co = 4, 3, 2
    X = RNG.standard_normal((ci, n, n, n))
    W = RNG.standard_normal((27, ci, co))
    b = RNG.standard_normal(co)
    Y = conv.conv3d(X, W, b)
    ref = np.zeros((co, n, n, n))
    for o in range(co):
        for a in range(n):
            for bb in range(n):
                for c in range(n):
                    s = b[o]
                    for t in range(27):
                        dx, dy, dz = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
                        for i in range(ci):
                            s += W[t, i, o] * X[i, (a + dx) % n, (bb + dy) % n,
                                                (c + dz) % n]
                    ref[o, a, bb, c] = s
    assert np.max(np.abs(Y - ref)) < 1e-12


def test_translation_equivariance():
    n = 6
    X = RNG.standard_normal((5, n, n, n))
    net = conv.Net.init(5, 4, width=8, seed=1)
    Y, _ = net.forward(X)
    Ys, _ = net.forward(np.roll(X, (1, 2, 3), axis=(1, 2, 3)))
    assert np.allclose(np.roll(Y, (1, 2, 3), axis=(1, 2, 3)), Ys, atol=1e-12)


@pytest.mark.parametrize("layer", [0, 2, 3])
def test_backward_matches_finite_differences(layer):
    n = 4
    X = RNG.standard_normal((3, n, n, n))
    T = RNG.standard_normal((2, n, n, n))
    net = conv.Net.init(3, 2, width=4, seed=layer + 10)
    # biases away from zero so that no ReLU sits at its kink
    net.params = [(W, b + 0.05 * RNG.standard_normal(b.shape))
                  for W, b in net.params]
    L, grads = net.loss_and_grads(X, T)
    W, b = net.params[layer]
    h = 1e-6
    for idx in [(0, 0, 0), (13, 1, 1), (26, 2, 0)]:
        idx = tuple(min(i, s - 1) for i, s in zip(idx, W.shape))
        Wp, Wm = W.copy(), W.copy()
        Wp[idx] += h
        Wm[idx] -= h
        ps = list(net.params)
        ps[layer] = (Wp, b)
        Lp = conv.Net(ps).loss_and_grads(X, T)[0]
        ps[layer] = (Wm, b)
        Lm = conv.Net(ps).loss_and_grads(X, T)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - grads[layer][0][idx]) < 1e-6 * max(1.0, abs(fd))
    j = 0
    bp, bm = b.copy(), b.copy()
    bp[j] += h
    bm[j] -= h
    ps = list(net.params)
    ps[layer] = (W, bp)
    Lp = conv.Net(ps).loss_and_grads(X, T)[0]
    ps[layer] = (W, bm)
    Lm = conv.Net(ps).loss_and_grads(X, T)[0]
    assert abs((Lp - Lm) / (2 * h) - grads[layer][1][j]) < 1e-6


def test_input_gradient_matches_finite_differences():
    n = 4
    X = RNG.standard_normal((2, n, n, n))
    W = RNG.standard_normal((27, 2, 3))
    b = RNG.standard_normal(3)
    dY = RNG.standard_normal((3, n, n, n))
    dX, _, _ = conv.conv3d_backward(X, W, dY)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 3, 2, 1)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[idx] += h
        Xm[idx] -= h
        fd = (np.sum(conv.conv3d(Xp, W, b) * dY)
              - np.sum(conv.conv3d(Xm, W, b) * dY)) / (2 * h)
        assert abs(fd - dX[idx]) < 1e-6 * max(1.0, abs(fd))


def test_adam_single_scalar():
    p = [(np.array([[[1.0]]]), np.array([0.5]))]
    g = [(np.array([[[0.2]]]), np.array([-0.1]))]
    st = {}
    out = conv.adam_step(p, g, st, lr=0.01)
    # first step: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps)
    assert np.isclose(out[0][0][0, 0, 0], 1.0 - 0.01 * 0.2 / (0.2 + 1e-8))
    assert np.isclose(out[0][1][0], 0.5 + 0.01 * 0.1 / (0.1 + 1e-8))
