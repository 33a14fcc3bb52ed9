"""FP64 reference of the warm-start network (oracle).

The network is not part of the paper; it predicts the fluctuation increment
of a load increment so that the Newton iteration of Sec. 2.1 (Eqs. 12-16)
starts closer to equilibrium.  Architecture: four 3x3x3 convolutions with
circular (periodic) padding, the same periodicity as the RVE of Eq. 1;
ReLU after the first three; channels in -> 32 -> 32 -> 32 -> out.

Conventions shared with the GPU kernels through the data, not the code:
* activations channels-first here, X[c, a, b, z] on the n^3 grid;
* tap t = (dx+1)*9 + (dy+1)*3 + (dz+1) for the offset (dx, dy, dz);
* weights W[t, c_in, c_out], bias b[c_out];
* Y[o, v] = b[o] + sum_t sum_i W[t, i, o] X[i, v + d_t]  (indices mod n).

Pins: forward against a voxel-by-voxel direct sum on a tiny grid, backward
against central finite differences, translation equivariance.  Status:
pinned.
"""

from __future__ import annotations

import numpy as np

OFFSETS = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1)
           for dz in (-1, 0, 1)]


def shift(X, d):
    """S[c, v] = X[c, v + d] on the periodic grid."""
    return np.roll(X, shift=(-d[0], -d[1], -d[2]), axis=(1, 2, 3))


def conv3d(X, W, b):
    """Circular 3x3x3 convolution: X (Ci, n, n, n) -> (Co, n, n, n)."""
    Co = W.shape[2]
    Y = np.broadcast_to(b.reshape(Co, 1, 1, 1), (Co,) + X.shape[1:]).copy()
    for t, d in enumerate(OFFSETS):
        Y += np.einsum("io,i...->o...", W[t], shift(X, d), optimize=True)
    return Y


def conv3d_backward(X, W, dY):
    """Gradients of conv3d: returns (dX, dW, db)."""
    dW = np.zeros_like(W)
    dX = np.zeros_like(X)
    for t, d in enumerate(OFFSETS):
        Xs = shift(X, d)
        dW[t] = np.einsum("i...,o...->io", Xs, dY, optimize=True)
        # dX[i, v + d] += W[t, i, o] dY[o, v]  ->  shift by -d
        dX += shift(np.einsum("io,o...->i...", W[t], dY, optimize=True),
                    (-d[0], -d[1], -d[2]))
    db = dY.sum(axis=(1, 2, 3))
    return dX, dW, db


class Net:
    """Four conv layers, ReLU after the first three."""

    def __init__(self, params):
        # params: list of (W, b)
        self.params = [(np.asarray(W, np.float64), np.asarray(b, np.float64))
                       for W, b in params]

    @staticmethod
    def init(cin, cout, width=32, seed=0, scale=1.0):
        rng = np.random.default_rng(seed)
        dims = [cin, width, width, width, cout]
        ps = []
        for i in range(4):
            fan = 27 * dims[i]
            W = rng.standard_normal((27, dims[i], dims[i + 1])) * np.sqrt(
                2.0 / fan) * (scale if i == 3 else 1.0)
            ps.append((W, np.zeros(dims[i + 1])))
        return Net(ps)

    def forward(self, X):
        acts = [X]
        zs = []
        h = X
        for k, (W, b) in enumerate(self.params):
            z = conv3d(h, W, b)
            zs.append(z)
            h = np.maximum(z, 0.0) if k < 3 else z
            acts.append(h)
        return h, (acts, zs)

    def loss_and_grads(self, X, T):
        """MSE over all outputs: L = mean((Y - T)^2)."""
        Y, (acts, zs) = self.forward(X)
        diff = Y - T
        L = float(np.mean(diff * diff))
        g = 2.0 * diff / diff.size
        grads = [None] * 4
        for k in range(3, -1, -1):
            if k < 3:
                g = g * (zs[k] > 0)
            dX, dW, db = conv3d_backward(acts[k], self.params[k][0], g)
            grads[k] = (dW, db)
            g = dX
        return L, grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015), in place; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    out = []
    for k, ((W, b), (dW, db)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((W, dW), (b, db))):
            key = (k, j)
            m = state.setdefault(("m",) + key, np.zeros_like(p))
            v = state.setdefault(("v",) + key, np.zeros_like(p))
            m[...] = b1 * m + (1 - b1) * g
            v[...] = b2 * v + (1 - b2) * g * g
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out
