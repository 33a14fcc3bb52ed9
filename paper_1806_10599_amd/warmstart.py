"""Training driver of the learned warm start (marshalling and bookkeeping).

The network's forward and backward passes, the loss and Adam run in the
HIP library (``rve_ws_*``); this module draws the initial parameters from a
seeded generator, collects (features, target) pairs from converged solver
increments, and loops over them.  Samples stay on the GPU as torch tensors
(device memory only; no arithmetic happens in torch).
"""

from __future__ import annotations

import os

import numpy as np

# parameters written by paper_1806_10599_amd.train_warmstart (float32 .npy)
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                       "warmstart.npy")

LAYERS = ((40, 32), (32, 32), (32, 32), (32, 9))


def param_count() -> int:
    return sum(27 * ci * co + co for ci, co in LAYERS)


def init_params(seed: int = 0, out_scale: float = 0.1) -> np.ndarray:
    """He-normal weights (last layer scaled by out_scale), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (ci, co) in enumerate(LAYERS):
        W = rng.standard_normal((27, ci, co)) * np.sqrt(2.0 / (27 * ci))
        if k == len(LAYERS) - 1:
            W *= out_scale
        parts += [W.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def trained_params(path: str = WEIGHTS) -> np.ndarray:
    """The shipped trained parameters (no pickled objects are loaded)."""
    p = np.load(path, allow_pickle=False)
    if p.dtype != np.float32 or p.shape != (param_count(),):
        raise ValueError(f"{path}: expected {param_count()} float32 parameters")
    return p


def unflatten(p):
    """Flat parameter vector -> [(W[27, cin, cout], b[cout]), ...]."""
    out, o = [], 0
    for ci, co in LAYERS:
        W = np.asarray(p[o:o + 27 * ci * co], dtype=np.float64).reshape(27, ci, co)
        o += 27 * ci * co
        b = np.asarray(p[o:o + co], dtype=np.float64)
        o += co
        out.append((W, b))
    return out


def collect(rve, history, max_samples=None, callback=None):
    """Run the solver over ``history``; keep (features, target, n) per
    converged increment that has a previous increment (the features need
    one)."""
    samples = []
    for j, inc in enumerate(history):
        if inc["cycle_start"]:
            rve.reset_fips()
        X = rve.features(inc["F_bar"]) if j > 0 else None
        info = rve.increment(inc["F_bar"], inc["dt"])
        if info["status"] != 0:
            raise RuntimeError(f"increment {inc['k']} failed ({info['status']})")
        if X is not None:
            samples.append((X, rve.target(), rve.n))
        if callback:
            callback(inc, info)
        if max_samples and len(samples) >= max_samples:
            break
    return samples


def train(net, samples, epochs=10, lr=1e-3, seed=0, log=None):
    """Adam over the samples in a seeded random order; returns the mean loss
    of each epoch."""
    rng = np.random.default_rng(seed)
    history = []
    for ep in range(epochs):
        order = rng.permutation(len(samples))
        tot = 0.0
        for i in order:
            X, T, n = samples[i]
            tot += net.train_step(X, T, n, lr)
        history.append(tot / max(1, len(samples)))
        if log:
            log(ep, history[-1])
    return history
