"""Train the learned warm start on converged increments of the synthetic
workloads and write its parameters.

    python -m paper_1806_10599_amd.train_warmstart \
        --out paper_1806_10599_amd/weights/warmstart.npy

Samples: every converged increment (after the first) of the 16^3 and 32^3
single-phase polycrystals and of the first four cycles of the 64^3
polycrystal with particles; the fifth 64^3 cycle is held out for
validation.  Each sample is the network input built from the committed
state before the increment and, as target, the part of the converged
fluctuation increment after it that the extrapolation of the one before
(scaled by the load ratio) misses (both produced by the library on the
GPU).  Training is Adam in the
library's kernels over the samples in a seeded order.  The held-out cycle
is then solved twice, with and without the network, and the predictor
residuals, Newton corrections and CG iterations are compared.

Writes the float32 parameter vector (``.npy``, loadable with
``numpy.load(..., allow_pickle=False)``) and a JSON report next to it.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def _workloads():
    from synthetic import config_by_name
    return [config_by_name("C1"), config_by_name("C2"), config_by_name("C3")]


def _rve(cfg, precision, warm_start=False, cg_forcing=0):
    from paper_1806_10599_amd.binding import Rve
    from synthetic import material_params
    micro = cfg.microstructure()
    r = Rve(micro.n, projection=cfg.operator, precision=precision,
            newton_tol=1e-6, cg_tol=1e-4, warm_start=warm_start,
            cg_forcing=cg_forcing)
    r.set_microstructure(micro.phase, micro.quat, micro.law, material_params())
    return r


def collect_all(log):
    """(train, validation) sample lists of (X, T, n) device tensors."""
    train, val = [], []
    for cfg in _workloads():
        hist = cfg.history()
        r = _rve(cfg, "mixed")
        t0 = time.perf_counter()
        for j, inc in enumerate(hist):
            if inc["cycle_start"]:
                r.reset_fips()
            X = r.features(inc["F_bar"]) if j > 0 else None
            info = r.increment(inc["F_bar"], inc["dt"])
            if info["status"] != 0:
                raise RuntimeError(f"{cfg.name} increment {j} failed")
            if X is None:
                continue
            sample = (X, r.target(), r.n)
            held_out = cfg.name == "C3" and inc["cycle"] == cfg.cycles - 1
            (val if held_out else train).append(sample)
        r.close()
        log(f"{cfg.name}: {len(hist)} increments in "
            f"{time.perf_counter() - t0:.1f} s")
    return train, val


def mean_loss(net, samples):
    return float(np.mean([net.loss(X, T, n) for X, T, n in samples]))


def evaluate(params_path_or_net, log):
    """Solve the held-out cycle with the homogeneous predictor, with the
    extrapolated start alone and with the network's correction of it (the
    benchmark's configuration: candidates kept directly when clearly
    better, inexact-Newton forcing mode 2)."""
    from synthetic import config_by_name
    cfg = config_by_name("C3")
    hist = cfg.history()
    first = next(j for j, inc in enumerate(hist) if inc["cycle"] == cfg.cycles - 1)
    out = {}
    for mode, ws in (("plain", 0), ("extrapolated", 3), ("learned", 2)):
        r = _rve(cfg, "mixed", warm_start=ws, cg_forcing=2)
        if mode == "learned":
            r.attach_warm_start(params_path_or_net)
        rows = []
        for j, inc in enumerate(hist):
            if inc["cycle_start"]:
                r.reset_fips()
            info = r.increment(inc["F_bar"], inc["dt"])
            if info["status"] != 0:
                raise RuntimeError(f"{mode}: increment {j} failed")
            if j >= first:
                rows.append(info)
        if mode == "learned":
            r.attach_warm_start(None)
        r.close()
        out[mode] = dict(
            newton=float(np.mean([i["newton_iters"] for i in rows])),
            cg=float(np.mean([i["cg_iters_total"] for i in rows])),
            predictor_residual=float(np.median([i["predictor_residual"] for i in rows])),
            plain_predictor_residual=float(np.median(
                [i["plain_predictor_residual"] for i in rows])),
            used_learned=float(np.mean([i["used_learned"] for i in rows])),
            sigma11=[float(i["sigma_bar"][0, 0]) for i in rows])
        log(f"held-out cycle, {mode}: Newton {out[mode]['newton']:.2f}, CG "
            f"{out[mode]['cg']:.1f} per increment, median predictor residual "
            f"{out[mode]['predictor_residual']:.3e}, learned start used in "
            f"{out[mode]['used_learned']:.0%} of increments")
    s_p = np.array(out["plain"]["sigma11"])
    s_l = np.array(out["learned"]["sigma11"])
    out["sigma11_max_rel_diff"] = float(np.max(np.abs(s_l - s_p)) / np.max(np.abs(s_p)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=os.path.join(
        os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart.npy"))
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)

    from paper_1806_10599_amd.binding import WarmStartNet
    from paper_1806_10599_amd.warmstart import init_params

    def log(msg):
        print(msg, flush=True)

    train, val = collect_all(log)
    log(f"{len(train)} training samples, {len(val)} held out")
    net = WarmStartNet()
    net.set_params(init_params(args.seed))
    rng = np.random.default_rng(args.seed)
    hist = []
    t0 = time.perf_counter()
    for ep in range(args.epochs):
        # geometric learning-rate decay from lr to lr_final
        frac = ep / max(1, args.epochs - 1)
        lr = args.lr * (args.lr_final / args.lr) ** frac
        order = rng.permutation(len(train))
        tr = float(np.mean([net.train_step(*train[i][:2], train[i][2], lr)
                            for i in order]))
        va = mean_loss(net, val)
        hist.append(dict(epoch=ep, lr=lr, train=tr, val=va))
        log(f"epoch {ep:3d} lr {lr:.2e} train {tr:.4e} val {va:.4e} "
            f"({time.perf_counter() - t0:.1f} s)")
    params = net.get_params()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, params.astype(np.float32), allow_pickle=False)
    ev = evaluate(net, log)
    report = dict(samples_train=len(train), samples_val=len(val),
                  epochs=args.epochs, lr=args.lr, lr_final=args.lr_final,
                  seed=args.seed, history=hist,
                  heldout={k: (v if k == "sigma11_max_rel_diff" else
                               {kk: vv for kk, vv in v.items() if kk != "sigma11"})
                           for k, v in ev.items()})
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(report, f, indent=1)
    net.close()
    log(f"wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
