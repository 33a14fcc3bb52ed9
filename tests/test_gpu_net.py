"""Warm-start network on the GPU against the FP64 oracle network.

bf16 weights and activations with FP32 accumulation are compared with the
FP64 reference element by element: on random weights within the bound of
bf16 rounding and FP32 accumulation that each element carries (the
reference uses the same bf16-rounded weights and inputs and rounds the
hidden activations to bf16 as the kernels do), and exactly on a network
whose arithmetic is exact in bf16 and FP32 (forward outputs bit for bit;
gradients within the bound of the bf16 rounding of the back-propagated
signal).  Also: training follows the oracle's Adam trajectory; the feature builder matches
its definition; a warm-started solve reaches the same equilibrium.
"""

import numpy as np
import pytest

from oracle import conv
from synthetic import config_by_name, macro_F

pytestmark = pytest.mark.gpu


def bf16_bits(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_round(x):
    return (bf16_bits(x).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _net(params):
    from paper_1806_10599_amd.binding import WarmStartNet
    net = WarmStartNet()
    net.set_params(params)
    return net


def _oracle_forward(params, X, emulate=True):
    """Reference forward with bf16-rounded weights; X (C, n, n, n)."""
    from paper_1806_10599_amd.warmstart import unflatten
    ps = [(bf16_round(W), b) for W, b in unflatten(params)]
    h = X
    acts = [X]
    for k, (W, b) in enumerate(ps):
        z = conv.conv3d(h, W, b)
        h = np.maximum(z, 0.0) if k < 3 else z
        if emulate and k < 3:
            h = bf16_round(h)
        acts.append(h)
    return h, ps


def _features(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n ** 3, 48)).astype(np.float32) * 0.5
    X[:, 40:] = 0.0
    bits = bf16_bits(X)
    Xt = torch.from_numpy(bits.view(np.int16).copy()).cuda()
    Xref = bf16_round(X)[:, :40].T.reshape(40, n, n, n)
    return Xt, Xref


GAMMA = 27 * 40 * 2.0 ** -24   # FP32 accumulation of one output (worst case)


def _forward_with_bound(ps, X):
    """Reference forward (bf16 weights ps, bf16-rounded hidden activations
    as the kernels do) and an element-wise bound on what the GPU may differ
    by: the FP32 accumulation of each output (GAMMA times the sum of
    |w||x|), a different rounding of a hidden activation to bf16 (one unit
    in the last place, 2^-7 |h|) and what the layers below already allowed,
    carried through |W|."""
    h, B = X, np.zeros_like(X)
    for k, (W, b) in enumerate(ps):
        z = conv.conv3d(h, W, b)
        M = conv.conv3d(np.abs(h), np.abs(W), np.abs(b))
        Bz = GAMMA * M + conv.conv3d(B, np.abs(W), np.zeros_like(b))
        if k == len(ps) - 1:
            return z, Bz
        h = bf16_round(np.maximum(z, 0.0))
        B = Bz * (1 + 2.0 ** -7) + 2.0 ** -7 * np.abs(h)


def test_forward_matches_oracle_elementwise():
    """Random weights and inputs: every output element within its bf16
    bound of the bf16-emulating FP64 reference."""
    from paper_1806_10599_amd.warmstart import init_params, unflatten
    n = 16
    p = init_params(3, out_scale=1.0)
    net = _net(p)
    Xt, Xref = _features(n, 1)
    Y = net.forward(Xt, n).cpu().numpy()
    net.close()
    ps = [(bf16_round(W), b) for W, b in unflatten(p)]
    ref, bound = _forward_with_bound(ps, Xref)
    ref, bound = ref.reshape(9, -1).T, bound.reshape(9, -1).T
    err = np.abs(Y[:, :9] - ref)
    print(f"max |gpu - ref| / bound {np.max(err / bound):.3f}, relative L2 "
          f"{np.linalg.norm(err) / np.linalg.norm(ref):.2e}")
    assert np.all(err <= bound)
    assert np.all(Y[:, 9:] == 0.0)


def _exact_net(seed, n):
    """Parameters and inputs whose whole forward pass is exact in bf16 and
    FP32: inputs in {-2, ..., 2}, about eight weights of +-1 per output,
    biases in {-0.5, 0, 0.5}; every hidden activation is then an integer or
    half-integer small enough for bf16 (checked)."""
    from paper_1806_10599_amd.warmstart import LAYERS
    rng = np.random.default_rng(seed)
    parts, ps = [], []
    for ci, co in LAYERS:
        W = rng.choice([-1.0, 1.0], size=(27, ci, co)) * (
            rng.random((27, ci, co)) < 8.0 / (27 * ci))
        b = rng.choice([-0.5, 0.0, 0.5], size=co)
        parts += [W.ravel(), b]
        ps.append((W, b))
    p = np.concatenate(parts).astype(np.float32)
    X = np.zeros((n ** 3, 48), dtype=np.float32)
    X[:, :40] = rng.integers(-2, 3, size=(n ** 3, 40))
    return p, ps, X


def test_forward_exact_arithmetic_matches_bit_for_bit():
    """A network whose arithmetic is exact in bf16 and FP32 gives the
    oracle's outputs exactly: any wrong tap, channel or sign shows."""
    import torch
    n = 16
    p, ps, X = _exact_net(11, n)
    Xref = X[:, :40].T.reshape(40, n, n, n).astype(np.float64)
    h = Xref
    for k, (W, b) in enumerate(ps):
        z = conv.conv3d(h, W, b)
        h = np.maximum(z, 0.0) if k < 3 else z
        if k < 3:
            assert np.array_equal(bf16_round(h), h), k   # exact in bf16
    ref = h.reshape(9, -1).T
    net = _net(p)
    Xt = torch.from_numpy(bf16_bits(X).view(np.int16).copy()).cuda()
    Y = net.forward(Xt, n).cpu().numpy()
    net.close()
    assert np.max(np.abs(ref)) > 4.0           # a non-trivial output
    assert np.array_equal(Y[:, :9].astype(np.float64), ref)


def test_gradients_match_oracle_elementwise():
    """Weight and bias gradients of all four layers (the weight-gradient
    kernel of each layer and the data-gradient path between them), on the
    exact-arithmetic network so that the forward pass agrees exactly: each
    element within the bound of the bf16 rounding of the back-propagated
    signal, (5 - k) 2^-7 times the sum of |x| |dY| over the same terms."""
    import torch
    n = 16
    p, ps, X = _exact_net(12, n)
    Xref = X[:, :40].T.reshape(40, n, n, n).astype(np.float64)
    rng = np.random.default_rng(9)
    T = np.zeros((n ** 3, 16), dtype=np.float32)
    T[:, :9] = rng.integers(-8, 9, size=(n ** 3, 9))
    Tt = torch.from_numpy(T).cuda()
    Xt = torch.from_numpy(bf16_bits(X).view(np.int16).copy()).cuda()
    net = _net(p)
    loss, g = net.train_step(Xt, Tt, n, lr=0.0, want_grad=True)
    assert np.array_equal(net.get_params(), p)   # lr = 0 changes nothing
    net.close()
    from paper_1806_10599_amd.warmstart import unflatten
    gu = unflatten(g)
    ref = conv.Net(ps)
    Y, (acts, zs) = ref.forward(Xref)
    Tr = T[:, :9].T.reshape(9, n, n, n).astype(np.float64)
    diff = Y - Tr
    Lref = float(np.mean(diff * diff))
    assert abs(loss - Lref) <= 1e-6 * Lref, (loss, Lref)
    gz = 2.0 * diff / diff.size
    G = np.abs(gz)
    worst = 0.0
    for k in range(3, -1, -1):
        if k < 3:
            gz = gz * (zs[k] > 0)
            G = G * (zs[k] > 0)
        W = ps[k][0]
        dX, dW, db = conv.conv3d_backward(acts[k], W, gz)
        dXa, dWa, dba = conv.conv3d_backward(np.abs(acts[k]), np.abs(W), G)
        c = (5 - k) * 2.0 ** -7
        for got, want, mag in ((gu[k][0], dW, dWa), (gu[k][1], db, dba)):
            err = np.abs(got - want)
            assert np.all(err <= c * mag + 1e-12), k
            nz = mag > 0
            worst = max(worst, float(np.max(err[nz] / (c * mag[nz]))))
        # the gradient is not identically zero where the bound is loose
        assert np.max(np.abs(dW)) > 0, k
        gz, G = dX, dXa
    print(f"max |gpu - ref| / bound over the gradients: {worst:.3f}")


def test_training_follows_the_oracle():
    """Forty Adam steps on the GPU track forty Adam steps of the FP64
    oracle network from the same parameters and data, step by step (the GPU
    rounds weights and activations to bf16, hence the 3 % tolerance), and
    the loss falls with the oracle's."""
    import torch
    from paper_1806_10599_amd.warmstart import init_params, unflatten
    n, steps, lr = 16, 40, 1e-3
    p = init_params(7)
    net = _net(p)
    Xt, Xref = _features(n, 3)
    # a target the network can represent: half the first nine input channels
    T = np.zeros((n ** 3, 16), dtype=np.float32)
    T[:, :9] = 0.5 * Xref[:9].reshape(9, -1).T
    Tt = torch.from_numpy(T).cuda()
    losses = [net.train_step(Xt, Tt, n, lr=lr) for _ in range(steps)]
    net.close()
    ref = conv.Net(unflatten(p))
    state, ref_losses = {}, []
    Tref = T[:, :9].T.reshape(9, n, n, n).astype(np.float64)
    for _ in range(steps):
        L, g = ref.loss_and_grads(Xref, Tref)
        ref_losses.append(L)
        ref.params = conv.adam_step(ref.params, g, state, lr=lr)
    # every step of the trajectory, and the oracle's own loss falls, so the
    # GPU's falls with it
    for k in range(steps):
        assert abs(losses[k] - ref_losses[k]) <= 0.03 * ref_losses[k], (
            k, losses[k], ref_losses[k])
    assert ref_losses[-1] < 0.85 * ref_losses[0], (ref_losses[0], ref_losses[-1])
    assert losses[-1] < 0.85 * losses[0], (losses[0], losses[-1])


def test_features_match_definition():
    from gpu_util import make_rve
    c = config_by_name("C1")
    micro = c.microstructure()
    hist = c.history()
    r = make_rve(micro, c.operator, "fp64")
    try:
        for inc in hist[:3]:
            Fprev = r.field("F")
            r.increment(inc["F_bar"], inc["dt"])
        F = r.field("F")
        dt_fluct = F - Fprev - (hist[2]["F_bar"] - hist[1]["F_bar"]).reshape(9, 1)
        dgam = r.field("dgamma")
        Fb3 = hist[3]["F_bar"]
        X = r.features(Fb3).cpu().numpy().view(np.uint16)
        Xf = (X.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        dF = (Fb3 - hist[2]["F_bar"]).ravel()
        dFp = (hist[2]["F_bar"] - hist[1]["F_bar"]).ravel()
        s, sp = np.linalg.norm(dF), np.linalg.norm(dFp)
        from oracle.crystal import quat_to_matrix
        R = np.array([quat_to_matrix(q).ravel() for q in micro.quat])
        ref = np.zeros((micro.n ** 3, 48))
        ref[:, 0:9] = dF / s
        ref[:, 9:18] = (dt_fluct / sp).T
        ref[:, 18:27] = 100 * (F - hist[2]["F_bar"].reshape(9, 1)).T
        ref[:, 27:36] = R[micro.phase]
        ref[:, 37] = dF @ dFp / (s * sp)
        ref[:, 38] = np.abs(dgam).sum(axis=0) / sp
        ref[:, 39] = 1.0
        assert np.allclose(Xf, bf16_round(ref), rtol=1e-2, atol=1e-6)
    finally:
        r.close()


def test_warm_start_keeps_the_equilibrium():
    from gpu_util import make_rve
    from paper_1806_10599_amd.warmstart import init_params
    c = config_by_name("C1")
    micro = c.microstructure()
    hist = c.history()[:6]
    net = _net(init_params(11, out_scale=0.01))
    a = make_rve(micro, c.operator, "mixed")
    b = make_rve(micro, c.operator, "mixed", warm_start=True)
    b.attach_warm_start(net)
    try:
        used = 0
        for inc in hist:
            ia = a.increment(inc["F_bar"], inc["dt"])
            ib = b.increment(inc["F_bar"], inc["dt"])
            assert ia["status"] == 0 and ib["status"] == 0
            assert ib["residual_rel"] <= 1e-6
            used += ib["used_learned"]
            s_a, s_b = ia["sigma_bar"][0, 0], ib["sigma_bar"][0, 0]
            assert abs(s_a - s_b) <= 1e-4 * abs(s_a) + 1e-3
        assert np.max(np.abs(a.field("F") - b.field("F"))) < 1e-4
    finally:
        b.attach_warm_start(None)
        a.close()
        b.close()
        net.close()


def test_loss_entry_point_leaves_training_state_alone():
    """rve_ws_loss returns the training step's loss and changes nothing."""
    import torch
    from paper_1806_10599_amd.warmstart import init_params
    n = 16
    p = init_params(2)
    a, b = _net(p), _net(p)
    Xt, Xref = _features(n, 4)
    T = np.zeros((n ** 3, 16), dtype=np.float32)
    T[:, :9] = 0.25 * Xref[9:18].reshape(9, -1).T
    Tt = torch.from_numpy(T).cuda()
    l0 = a.loss(Xt, Tt, n)
    assert a.loss(Xt, Tt, n) == l0
    for _ in range(3):
        la = a.train_step(Xt, Tt, n, lr=1e-3)
        b.loss(Xt, Tt, n)          # interleaved evaluations
        lb = b.train_step(Xt, Tt, n, lr=1e-3)
        assert la == lb
    assert l0 == _net(p).train_step(Xt, Tt, n, lr=0.0)
    assert np.array_equal(a.get_params(), b.get_params())
    a.close()
    b.close()


def test_shipped_weights_beat_the_homogeneous_predictor_on_held_out_cycle():
    """The trained parameters (never trained on the fifth 64^3 cycle) give a
    smaller predictor residual there and the same equilibrium."""
    from gpu_util import make_rve
    from paper_1806_10599_amd.warmstart import trained_params
    c = config_by_name("C3")
    micro = c.microstructure()
    hist = c.history()
    first = next(j for j, inc in enumerate(hist) if inc["cycle"] == c.cycles - 1)
    stop = first + 10
    net = _net(trained_params())
    a = make_rve(micro, c.operator, "mixed")
    b = make_rve(micro, c.operator, "mixed", warm_start=True)
    b.attach_warm_start(net)
    try:
        ra, rb = [], []
        for j, inc in enumerate(hist[:stop]):
            if inc["cycle_start"]:
                a.reset_fips()
                b.reset_fips()
            ia = a.increment(inc["F_bar"], inc["dt"])
            ib = b.increment(inc["F_bar"], inc["dt"])
            assert ia["status"] == 0 and ib["status"] == 0
            if j >= first:
                ra.append(ia)
                rb.append(ib)
        used = np.mean([i["used_learned"] for i in rb])
        pa = np.median([i["predictor_residual"] for i in ra])
        pb = np.median([i["predictor_residual"] for i in rb])
        assert used >= 0.8, used
        assert pb < 0.5 * pa, (pa, pb)
        for x, y in zip(ra, rb):
            s_a, s_b = x["sigma_bar"][0, 0], y["sigma_bar"][0, 0]
            assert abs(s_a - s_b) <= 1e-4 * abs(s_a) + 1e-3
    finally:
        b.attach_warm_start(None)
        a.close()
        b.close()
        net.close()


def test_direct_acceptance_mode_keeps_clearly_better_candidates():
    """warm_start = 2: a learned candidate whose FP64 residual is below half
    of the homogeneous predictor's last evaluated residual is kept without
    evaluating the homogeneous predictor; otherwise both are evaluated as in
    mode 1.  The equilibrium is the same as without the network."""
    from gpu_util import make_rve
    from paper_1806_10599_amd.warmstart import trained_params
    c = config_by_name("C3")
    micro = c.microstructure()
    hist = c.history()[:50]
    net = _net(trained_params())
    a = make_rve(micro, c.operator, "mixed")
    b = make_rve(micro, c.operator, "mixed", warm_start=2)
    b.attach_warm_start(net)
    try:
        last_plain = None
        direct = 0
        for j, inc in enumerate(hist):
            if inc["cycle_start"]:
                a.reset_fips()
                b.reset_fips()
            ia = a.increment(inc["F_bar"], inc["dt"])
            ib = b.increment(inc["F_bar"], inc["dt"])
            assert ia["status"] == 0 and ib["status"] == 0
            s_a, s_b = ia["sigma_bar"][0, 0], ib["sigma_bar"][0, 0]
            assert abs(s_a - s_b) <= 1e-4 * abs(s_a) + 1e-3
            if ib["plain_predictor_residual"] < 0:
                direct += 1
                assert ib["used_learned"] == 1 and last_plain is not None
                assert ib["predictor_residual"] < 0.5 * last_plain
            else:
                last_plain = ib["plain_predictor_residual"]
        assert direct >= 0.5 * len(hist), direct
    finally:
        b.attach_warm_start(None)
        a.close()
        b.close()
        net.close()


def test_learned_correction_beats_the_extrapolated_start_on_held_out_cycle():
    """The network predicts the correction to the extrapolated start (last
    fluctuation increment x load ratio, warm_start = 3); on the held-out
    fifth 64^3 cycle, in the benchmark's configuration (direct acceptance,
    forcing mode 2), the corrected start needs fewer Newton corrections and
    CG iterations than the extrapolation alone, at the same equilibrium."""
    from gpu_util import make_rve
    from paper_1806_10599_amd.warmstart import trained_params
    c = config_by_name("C3")
    micro = c.microstructure()
    hist = c.history()
    first = next(j for j, inc in enumerate(hist) if inc["cycle"] == c.cycles - 1)
    net = _net(trained_params())
    a = make_rve(micro, c.operator, "mixed", warm_start=3, cg_forcing=2)
    b = make_rve(micro, c.operator, "mixed", warm_start=2, cg_forcing=2)
    b.attach_warm_start(net)
    try:
        ra, rb = [], []
        for j, inc in enumerate(hist):
            if inc["cycle_start"]:
                a.reset_fips()
                b.reset_fips()
            ia = a.increment(inc["F_bar"], inc["dt"])
            ib = b.increment(inc["F_bar"], inc["dt"])
            assert ia["status"] == 0 and ib["status"] == 0
            if j >= first:
                ra.append(ia)
                rb.append(ib)
        na = sum(i["newton_iters"] for i in ra)
        nb = sum(i["newton_iters"] for i in rb)
        ca = sum(i["cg_iters_total"] for i in ra)
        cb = sum(i["cg_iters_total"] for i in rb)
        print(f"held-out cycle: extrapolated Newton {na} CG {ca}, "
              f"learned Newton {nb} CG {cb}")
        assert nb <= na and cb < ca
        for x, y in zip(ra, rb):
            s_a, s_b = x["sigma_bar"][0, 0], y["sigma_bar"][0, 0]
            assert abs(s_a - s_b) <= 1e-5 * abs(s_a) + 1e-3
    finally:
        b.attach_warm_start(None)
        a.close()
        b.close()
        net.close()
