"""Benchmark: Newton-converged voxel-increments/s at 64^3 (chosen vs plain).

Workload: the 64^3 RVE (200 Voronoi grains plus 8 % stiff particles,
discrete projection operator, five fully reversed +-0.6 % cycles of 40
increments), synthetic and seeded.  One "step" is one load increment of
that RVE solved to equilibrium tolerance 1e-6 (FP64 residual): predictor,
return mapping, residual, Newton-CG, commit.  The timed steps are the last
``--steps`` increments of the history (by default the fifth cycle, which the
warm-start network never saw in training); the increments before them run
untimed to reach that state.

* chosen: FP32 FFT/projection/CG, FP64 return mapping/residual/averages,
  learned warm start (the shipped network's correction to the extrapolated
  fluctuation increment, kept at once when well below the homogeneous
  predictor's last residual, with the homogeneous predictor as fallback),
  inexact-Newton forcing (mode 2), CG schedule tuned on the live buffers.
  Direct launches: replaying the CG chunks from captured graphs (--graph)
  measures the same rate here, and direct launches let each timed kernel
  record its own start and end.
* plain:  FP64 everywhere, direct launches, same kernels, same inputs.

``value`` is the chosen path's voxel-increments/s.  Inside its timed region
every launch of the hot-path kernels is bracketed by HIP events on the
solver's stream (CG graphs included), so the JSON line carries each
kernel's live average duration, the roofline of the dominant kernel (by
total time), the plain path, and the CPU oracle timed on a bounded sample
of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Newton-converged voxel-increments/s at 64^3 (chosen vs plain, "
          "tol 1e-6); FFT GB/s")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# algorithmic HBM bytes per voxel of each CG-iteration kernel on the FP32
# path (each datum read or written once; the packed half spectrum of nine
# components is 9 x n^3/2 complex = 36 B per voxel)
PASS_BYTES_F32 = {
    # K (81 floats), r, p_old, x in; p, K:p, x out (the previous iteration's
    # x += alpha p_old rides on the direction kernel)
    "matvec_kp": 4 * (81 + 9 + 9 + 9 + 9 + 9 + 9),
    "matvec_pass_a": 4 * 9 + 36,                    # K:p in, half spectrum out
    "matvec_pass_b": 36 + 36,                       # spectrum in and out
    "matvec_pass_c": 36 + 4 * 9 + 4 * 9,            # spectrum, r in; r out
}
# the same with the direction step and K:p folded into pass A (fused
# schedule): K, r, p_old, x in; p, x, half spectrum out; no K:p round trip
PASS_BYTES_F32_FUSED = {
    "matvec_pass_a": 4 * (81 + 9 + 9 + 9 + 9 + 9) + 36,
    "matvec_pass_b": 36 + 36,
    "matvec_pass_c": 36 + 4 * 9 + 4 * 9,
}


def pass_bytes(fused):
    return PASS_BYTES_F32_FUSED if fused else PASS_BYTES_F32


def live_classes(fused):
    """Kernel classes timed live in the timed region: the return mapping and
    the K:p kernel (pass A when K:p is folded into it)."""
    return LIVE_CLASSES[:1] + (("matvec_pass_a",) if fused else ("matvec_kp",))
# algorithmic flops of the return mapping (add, mul, div, sqrt and each
# elementary function count 1, a fused multiply-add 2; counted once per voxel
# from the algorithm, not from the instruction stream), FP64 and FP32 apart:
# per residual evaluation (plastic and elastic deformation, stress, 12
# resolved shears, back stresses, the one-logarithm residuals; FP32 flow
# slopes), per local Newton step (FP32 Jacobian: 12 rank-one updates of the
# 6x6 capacitance matrix, its LU factorisation, the Woodbury solve; FP64
# step and convergence tests), per crystal voxel (set-up, final Fp^-1 and
# P) and per particle voxel
RM_FLOPS = {"eval64": 1206, "eval32": 72, "step64": 60, "step32": 2350,
            "crystal64": 825, "particle64": 90}
# kernel classes timed live in the timed region: the K:p direction kernel
# (the dominant kernel, on a sample of its launches) and the return mapping
# (every launch: its ALU roofline needs the local Newton steps of the same
# launches).  Every class, the tangent, the FP64 residual and the three FFT
# passes included, is timed on every launch over the sample increments
# before the timed region: an event pair costs 12-18 us of the stream's
# time, and timing the tangent and the residual in the timed region as well
# cost 1.2 % of the throughput.
LIVE_CLASSES = ("return_map", "matvec_kp")
# the K:p kernel (one launch per CG iteration) is timed on one launch in
# 29 in the timed region (about 120 timed launches over the 40 timed
# increments): an event pair on every launch cost about 8 % of the
# throughput, one in seven about 1 %; 29 is prime to every CG chunk length
# (1 to 8), so the sample walks through every position of a chunk
LIVE_CG_STRIDE = 29
# learned warm start: a candidate well below the homogeneous predictor's
# last residual is kept without evaluating the homogeneous predictor
WARM_MODE = 2
# inexact-Newton forcing mode of the chosen path (set from --forcing-mode)
FORCING = 2


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-live", action="store_true",
                    help="no live kernel timing (no events in the timed region)")
    ap.add_argument("--live-cg-stride", type=int, default=LIVE_CG_STRIDE,
                    help="time one K:p launch in this many in the timed region")
    ap.add_argument("--start", type=int, default=None,
                    help="first timed increment (0-based; default: the last "
                         "--steps increments of the history are timed)")
    ap.add_argument("--cg-chunk", type=int, default=8,
                    help="CG iterations between host convergence checks")
    ap.add_argument("--no-learned", action="store_true",
                    help="chosen path without the learned warm start")
    ap.add_argument("--graph", action="store_true",
                    help="chosen path replays CG chunks from captured graphs "
                         "(live timing then uses event-record nodes)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-RVE measurement")
    ap.add_argument("--batch-steps", type=int, default=8)
    ap.add_argument("--large-steps", type=int, default=6,
                    help="increments of the 128^3 RVE (0: skip)")
    ap.add_argument("--paper-workloads", action="store_true",
                    help="also run the paper's own R = 0 histories (a few "
                         "minutes)")
    ap.add_argument("--fft-schedule", default=None,
                    help="force the CG-matvec FFT schedule of the chosen path "
                         "as CPB,TT (e.g. 1,8) instead of tuning it; counter "
                         "runs serialize kernels, which makes tuning there "
                         "meaningless")
    ap.add_argument("--forcing-mode", type=int, default=2, choices=(1, 2),
                    help="inexact-Newton forcing of the chosen, batch and "
                         "128^3 paths (1: only as tight as a quarter of the "
                         "equilibrium tolerance needs; 2: half of it, and "
                         "never tighter than 0.05 of the residual)")
    ap.add_argument("--no-forcing", action="store_true",
                    help="chosen path solves every Newton iteration to "
                         "cg_tol (no inexact-Newton forcing)")
    ap.add_argument("--no-umat", action="store_true",
                    help="skip the Appendix A bridge measurement")
    ap.add_argument("--no-ablations", action="store_true",
                    help="skip the ablation rows (forcing, precision, "
                         "extrapolated start) of the chosen path")
    ap.add_argument("--no-paper-case", action="store_true",
                    help="skip the paper's Sec. 5 case on 32^3 (three R = 0 "
                         "cycles at 1 %%, chosen and FP64 paths)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain elementwise copy of 256 MiB "
                         "(read + write), the reference kernel that scales "
                         "hardware byte counters")
    return ap.parse_args()


def copy_bandwidth(stream, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth on this GPU: a plain device-to-device copy of
    nbytes (read + write counted), timed with events on the stream."""
    import torch
    with torch.cuda.stream(stream):
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(
            enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.copy_(a)
        e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return round(2 * nbytes / sec / 1e9, 1)


def copy_calibration(stream):
    """A plain copy kernel of known size: reads and writes 2^26 floats."""
    import torch
    with torch.cuda.stream(stream):
        x = torch.ones(1 << 26, device="cuda", dtype=torch.float32)
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    return {"kernel": "elementwise mul by 1 (torch)", "bytes_read": 1 << 28,
            "bytes_written": 1 << 28}


def run_path(micro, hist, precision, use_graph, steps, warmup, stream,
             live=True, learned=False, start=None, cg_chunk=8,
             with_fips=False, forcing=False, schedule=None, check=False,
             sample_all=False, warm_start=None):
    """Solve the history; time its last ``steps`` increments (at least
    ``warmup`` untimed increments come first).

    check: the committed state before the last timed increment and the
    fields after it are copied out (outside the timed region: the K steps
    are timed as two bracketed intervals, increments 1..K-1 and K) for the
    oracle's error checks.  sample_all: the two increments before the timed
    window run with every hot-path kernel class timed live (the CG kernels
    included), to rank the kernels by their share of an increment."""
    import torch
    from paper_1806_10599_amd.binding import (KERNEL_CLASSES, Rve,
                                              WarmStartNet)
    from paper_1806_10599_amd.warmstart import trained_params
    from synthetic import material_params
    ws = (WARM_MODE if learned else 0) if warm_start is None else warm_start
    r = Rve(micro.n, projection="discrete", precision=precision,
            newton_tol=1e-6, cg_tol=1e-4, use_graph=use_graph, stream=stream,
            warm_start=ws, cg_chunk=cg_chunk, cg_forcing=forcing)
    r.set_microstructure(micro.phase, micro.quat, micro.law, material_params())
    if schedule:
        r.set_fft_schedule(*schedule)
    net = None
    if learned:
        net = WarmStartNet(stream=stream)
        net.set_params(trained_params())
        r.attach_warm_start(net)
    start = max(warmup, len(hist) - steps) if start is None else max(warmup, start)
    sample, sample_cg = None, 0
    for j, inc in enumerate(hist[:start]):
        if sample_all and j == start - 2:
            torch.cuda.synchronize()
            r.set_kernel_timing(KERNEL_CLASSES)
            r.kernel_timing(reset=True)
        if inc["cycle_start"]:
            r.reset_fips()
        info = r.increment(inc["F_bar"], inc["dt"])
        if info["status"] != 0:
            raise RuntimeError(f"increment {inc['k']} failed: {info['status']}")
        if sample_all and j >= start - 2:
            sample_cg = sample_cg + info["cg_iters_total"]
    if sample_all:
        torch.cuda.synchronize()
        sample = dict(increments=[int(hist[start - 2]["k"]),
                                  int(hist[start - 1]["k"])],
                      timing=r.kernel_timing(reset=True), cg_total=sample_cg)
        r.set_kernel_timing(())
    fused = bool(r.fft_schedule()["fused"])
    if live:
        r.set_kernel_timing(live_classes(fused), cg_stride=LIVE_CG_STRIDE)
    torch.cuda.synchronize()
    r.kernel_timing(reset=True)
    r.return_map_counts(reset=True)
    window = hist[start:start + steps]
    timed = []
    chk = None
    elapsed = 0.0
    parts = [window[:-1], window[-1:]] if check else [window]
    for part in parts:
        if check and part is parts[1]:
            before = r.fields("Fpinv", "chi")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for inc in part:
            if inc["cycle_start"]:
                r.reset_fips()
            info = r.increment(inc["F_bar"], inc["dt"])
            if info["status"] != 0:
                raise RuntimeError(f"increment {inc['k']} failed: "
                                   f"{info['status']}")
            timed.append(info)
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
    if check:
        after = r.fields("F", "P", "dgamma")
        inc = window[-1]
        chk = dict(k=int(inc["k"]), F_bar=np.asarray(inc["F_bar"]),
                   dt=inc["dt"], Fpi0=before["Fpinv"], chi0=before["chi"],
                   F=after["F"], P=after["P"], dg=after["dgamma"],
                   residual_rel=timed[-1]["residual_rel"])
    live_t = r.kernel_timing() if live else None
    seen = r.kernel_launches() if live else None
    counts = r.return_map_counts() if live else None
    sched = r.fft_schedule()
    nonlocal_ = nonlocal_fips_report(r, micro.n) if with_fips else None
    passes = (cg_pass_report(r.bench_kernels(reps=50), micro.n ** 3,
                             sched["fused"])
              if precision == "mixed" and with_fips else None)
    sig = [i["sigma_bar"][0, 0] for i in timed]
    if net is not None:
        r.attach_warm_start(None)
        net.close()
    r.close()
    return dict(elapsed=elapsed, infos=timed, live=live_t, seen=seen,
                rm_counts=counts,
                sigma11=sig, schedule=sched, start=start, nonlocal_=nonlocal_,
                passes=passes, check=chk, sample=sample)


def cg_pass_report(kern, N, fused=False):
    """Achieved bandwidth of the CG-iteration kernels (FP32) from
    back-to-back launches with the solver's launch configuration and the
    tuned FFT schedule, on the buffers of the last increment (after the
    timed window): algorithmic bytes per launch / average duration."""
    out = {}
    pb = pass_bytes(fused)
    for k, b in pb.items():
        ms = kern[k]
        gbs = N * b / (ms * 1e-3) / 1e9
        out[k] = dict(us=round(1e3 * ms, 2), bytes_per_voxel=b,
                      gbps=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 3))
    mv = ("matvec_pass_a", "matvec_pass_b", "matvec_pass_c")
    ms = sum(kern[k] for k in mv)
    gbs = N * sum(pb[k] for k in mv) / (ms * 1e-3) / 1e9
    out["fft_projection_passes"] = dict(us=round(1e3 * ms, 2), gbps=round(gbs, 1),
                                        frac=round(gbs / HBM_PEAK_GBS, 3))
    if fused:
        out["fft_projection_passes"]["includes"] = "direction step and K:p (pass A)"
    ms_all = sum(kern[k] for k in pb)
    out["cg_iteration_us"] = round(1e3 * ms_all, 2)
    return out


def nonlocal_fips_report(r, n, width_voxels=2.0):
    """Eqs. 25-26 on the committed indicator fields (after the timed
    window): the first call builds the band lists on the host, later calls
    only run the device reductions."""
    import torch
    w = width_voxels / n
    t0 = time.perf_counter()
    first = r.nonlocal_fips(w, arrays=False)
    t1 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        res = r.nonlocal_fips(w, arrays=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    assert res["wcyc_b"] == first["wcyc_b"]
    return {"band_width_voxels": width_voxels, "grains": res["grains"],
            "bands": res["bands"], "pcyc_g": res["pcyc_g"],
            "pcyc_lit_g": res["pcyc_lit_g"], "wcyc_b": res["wcyc_b"],
            "first_call_ms": round(1e3 * (t1 - t0), 3),
            "call_ms": round(1e3 * (t2 - t1) / reps, 3)}


def batch_run(steps, stream):
    """The batch workload: 32 RVEs of edges 24-48 (20-150 grains each, about
    1.8 M voxels), one launch per pass for the whole batch with a CG
    schedule tuned per edge and the host checking each CG chunk; the same
    batch with the device-controlled increment (one persistent launch per
    linear solve, captured graph); then the same RVEs and increments solved
    one after another with single-RVE handles (same precision, operator and
    tolerances).  All timed over the first ``steps`` increments, schedules
    tuned beforehand."""
    import torch
    from paper_1806_10599_amd.binding import BatchRve, Rve
    from synthetic import config_by_name, material_params
    cfg = config_by_name("C4")
    micros = cfg.batch_microstructures()
    hist = cfg.history()[:steps]
    vox = sum(m.n ** 3 for m in micros)
    b = BatchRve([m.n for m in micros], projection=cfg.operator,
                 precision=cfg.precision, newton_tol=1e-6, cg_tol=1e-4,
                 use_graph=False, stream=stream, cg_forcing=FORCING)
    for j, m in enumerate(micros):
        b.set_microstructure(j, m.phase, m.quat, m.law, material_params())
    b.tune_fft_schedules()   # per edge, outside the timed increments
    newton = []
    t_batch = 0.0
    # timed as two bracketed intervals (increments 1..K-1 and K) so that
    # RVE 0's committed state before the last one can be copied out for
    # the oracle's error checks
    for pi, part in enumerate((hist[:-1], hist[-1:])):
        if pi == 1:
            before = {f: b.field(0, f) for f in ("Fpinv", "chi")}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for inc in part:
            infos = b.increment(inc["F_bar"], inc["dt"])
            if any(i["status"] != 0 for i in infos):
                raise RuntimeError("batched increment failed")
            newton.append(max(i["newton_iters"] for i in infos))
        torch.cuda.synchronize()
        t_batch += time.perf_counter() - t0
    chk = dict(k=int(hist[-1]["k"]), F_bar=np.asarray(hist[-1]["F_bar"]),
               dt=hist[-1]["dt"], Fpi0=before["Fpinv"], chi0=before["chi"],
               F=b.field(0, "F"), P=b.field(0, "P"), dg=b.field(0, "dgamma"),
               residual_rel=infos[0]["residual_rel"])
    sig_b = [b.macro(j)["sigma_bar"][0, 0] for j in range(len(micros))]
    scheds = {str(e): v for e, v in b.fft_schedules().items()}
    # statistical volume element: Eqs. 25-26 per RVE, mean and standard
    # deviation over the RVEs (bands two voxel edges wide)
    fb = [b.nonlocal_fips(j, arrays=False) for j in range(len(micros))]
    pg = np.array([f["pcyc_g"] for f in fb])
    wb = np.array([f["wcyc_b"] for f in fb])
    sve = {"rves": len(fb), "band_width_voxels": 2.0,
           "pcyc_g_mean": float(pg.mean()), "pcyc_g_std": float(pg.std(ddof=1)),
           "wcyc_b_mean": float(wb.mean()), "wcyc_b_std": float(wb.std(ddof=1))}
    b.close()
    # the same batch with the Newton decisions on the device, each linear
    # solve of all RVEs in one persistent launch (grid barriers between the
    # passes) and the predictor and first Newton iterations replayed from a
    # captured graph
    bd = BatchRve([m.n for m in micros], projection=cfg.operator,
                  precision=cfg.precision, newton_tol=1e-6, cg_tol=1e-4,
                  use_graph=True, stream=stream, cg_forcing=FORCING)
    for j, m in enumerate(micros):
        bd.set_microstructure(j, m.phase, m.quat, m.law, material_params())
    bd.tune_fft_schedules()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for inc in hist:
        if any(i["status"] != 0 for i in bd.increment(inc["F_bar"], inc["dt"])):
            raise RuntimeError("device-controlled batched increment failed")
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    sig_d = np.array([bd.macro(j)["sigma_bar"][0, 0] for j in range(len(micros))])
    bd.close()
    t_single = 0.0
    sig_s = []
    for m in micros:
        r = Rve(m.n, projection=cfg.operator, precision=cfg.precision,
                newton_tol=1e-6, cg_tol=1e-4, stream=stream, cg_forcing=FORCING)
        r.set_microstructure(m.phase, m.quat, m.law, material_params())
        r.tune_fft_schedule()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for inc in hist:
            if r.increment(inc["F_bar"], inc["dt"])["status"] != 0:
                raise RuntimeError("single-RVE increment failed")
        torch.cuda.synchronize()
        t_single += time.perf_counter() - t0
        sig_s.append(r.macro()["sigma_bar"][0, 0])
        r.close()
    sig_b, sig_s = np.array(sig_b), np.array(sig_s)
    return {"workload": (f"{len(micros)} RVEs, edges "
                         f"{sorted(set(m.n for m in micros))}, {vox} voxels, "
                         f"{cfg.operator} operator, {cfg.precision}, tol 1e-6, "
                         f"first {steps} increments of +-{cfg.eps_a:.1%} cycles"),
            "value": round(vox * steps / t_batch, 1),
            "unit": "voxel-increments/s",
            "ms_per_step": round(1e3 * t_batch / steps, 3),
            "max_newton_per_increment": float(np.mean(newton)),
            "launches": ("one launch per pass for the whole batch, Newton "
                         "decisions and CG chunk checks on the host"),
            "fft_schedules": scheds,
            "persistent_graph": {
                "persistent": True,
                "graph": ("predictor and the first four Newton iterations "
                          "replayed from one captured graph per increment; "
                          "Newton decisions on the device; each linear solve "
                          "of all RVEs one persistent launch with grid "
                          "barriers between the passes"),
                "ms_per_step": round(1e3 * t_dev / steps, 3),
                "value": round(vox * steps / t_dev, 1),
                "over_one_launch_per_pass": round(t_batch / t_dev, 3),
                "sigma11_max_rel_diff": float(
                    np.max(np.abs(np.array(sig_b) - sig_d))
                    / np.max(np.abs(np.array(sig_b))))},
            "one_by_one_value": round(vox * steps / t_single, 1),
            "batched_over_one_by_one": round(t_single / t_batch, 3),
            "sigma11_max_rel_diff_vs_one_by_one": float(
                np.max(np.abs(sig_b - sig_s)) / np.max(np.abs(sig_s))),
            "sve_nonlocal_fips": sve,
            "_check": chk, "_micro0": micros[0]}


def large_run(steps, stream):
    """The 128^3 RVE (1000 grains, 5 % particles, never seen by the
    warm-start training): its first ``steps`` increments with the learned
    start and, for comparison, with the homogeneous predictor; both mixed
    precision.  The first increment has no history for the network and is
    left out of the statistics."""
    import torch
    from synthetic import config_by_name
    cfg = config_by_name("C5")
    micro = cfg.microstructure()
    hist = cfg.history()[:steps]
    out = {"workload": (f"{cfg.n}^3 RVE, {cfg.grains} grains + "
                        f"{cfg.particle_fraction:.0%} stiff particles, "
                        f"{cfg.operator} operator, mixed, tol 1e-6, increments "
                        f"2-{steps} of +-{cfg.eps_a:.1%} cycles")}
    for mode in ("learned", "homogeneous"):
        r = run_path(micro, hist, "mixed", False, steps - 1, 1, stream,
                     live=False, learned=(mode == "learned"), start=1,
                     with_fips=(mode == "learned"), forcing=FORCING,
                     check=(mode == "learned"))
        if r["check"] is not None:
            out["_check"], out["_micro"] = r["check"], micro
        n3 = micro.n ** 3
        out[mode] = dict(value=round(n3 * (steps - 1) / r["elapsed"], 1),
                         ms_per_step=round(1e3 * r["elapsed"] / (steps - 1), 3),
                         **predictor_stats(r["infos"]))
        if r["passes"]:
            out["cg_passes"] = r["passes"]
    out["unit"] = "voxel-increments/s"
    return out


# Appendix A bridge: FP64 reads F (9), sigma (6), ddsdde (36) and writes
# P (9), K (81) per voxel
UMAT_BYTES = 8 * (9 + 6 + 36 + 9 + 81)


def umat_run(stream, n=128 ** 3, calls=20):
    """The Appendix A bridge on n voxels of a user material's output (Cauchy
    stress and Jaumann-rate tangent): mean duration of one call from HIP
    events on the launch stream, against HBM bandwidth."""
    import torch
    from paper_1806_10599_amd.binding import umat_bridge
    g = torch.Generator(device="cuda").manual_seed(0)
    with torch.cuda.stream(stream):
        F = torch.eye(3, dtype=torch.float64, device="cuda").reshape(9, 1) + \
            0.15 * torch.randn((9, n), dtype=torch.float64, device="cuda",
                               generator=g)
        sig = torch.randn((6, n), dtype=torch.float64, device="cuda", generator=g)
        D = torch.randn((36, n), dtype=torch.float64, device="cuda", generator=g)
        umat_bridge(F, sig, D, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(
            enable_timing=True)
        e0.record(stream)
        for _ in range(calls):
            umat_bridge(F, sig, D, stream)
        e1.record(stream)
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / calls
    gbs = UMAT_BYTES * n / (us * 1e-6) / 1e9
    return {"workload": f"{n} voxels, FP64 (F, sigma, 6x6 tangent -> P, K)",
            "us_per_call": round(us, 2), "bytes_per_voxel": UMAT_BYTES,
            "voxels_per_s": round(n / (us * 1e-6), 1),
            "achieved_GBps": round(gbs, 1), "peak_GBps": HBM_PEAK_GBS,
            "frac": round(gbs / HBM_PEAK_GBS, 3)}


def _eq29_per_cycle(sig, ref, per_cycle):
    """Eq. 29 (max over each cycle of |sigma - sigma_ref| / max |sigma_ref|,
    in %), one value per cycle."""
    sig, ref = np.asarray(sig), np.asarray(ref)
    scale = np.max(np.abs(ref))
    d = np.abs(sig - ref) / scale * 100.0
    return [float(np.max(d[c:c + per_cycle])) for c in range(0, len(d), per_cycle)]


def _run_history(micro, hist, precision, operator, stream, adaptive=False,
                 learned=False, forcing=False):
    """Solve a whole history; returns seconds, sigma_11 per increment and
    solver counts."""
    import torch
    from paper_1806_10599_amd.binding import Rve, WarmStartNet
    from paper_1806_10599_amd.warmstart import trained_params
    from synthetic import material_params
    r = Rve(micro.n, projection=operator, precision=precision,
            newton_tol=1e-6, cg_tol=1e-4, stream=stream,
            warm_start=WARM_MODE if learned else 0, cg_forcing=forcing)
    r.set_microstructure(micro.phase, micro.quat, micro.law, material_params())
    net = None
    if learned:
        net = WarmStartNet(stream=stream)
        net.set_params(trained_params())
        r.attach_warm_start(net)
    sig, newton, cg, sub, cuts = [], 0, 0, 0, 0
    r.tune_fft_schedule()   # outside the timed history
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for inc in hist:
        if inc["cycle_start"]:
            r.reset_fips()
        if adaptive:
            a = r.increment_adaptive(inc["F_bar"], inc["dt"], max_cutbacks=6)
            if a["status"] != 0:
                raise RuntimeError(f"increment {inc['k']} failed: {a['status']}")
            newton += a["newton_iters_total"]
            cg += a["cg_iters_total"]
            sub += a["substeps"]
            cuts += a["cutbacks"]
            sig.append(a["last"]["sigma_bar"][0, 0])
        else:
            info = r.increment(inc["F_bar"], inc["dt"])
            if info["status"] != 0:
                raise RuntimeError(f"increment {inc['k']} failed: {info['status']}")
            newton += info["newton_iters"]
            cg += info["cg_iters_total"]
            sig.append(info["sigma_bar"][0, 0])
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    if net is not None:
        r.attach_warm_start(None)
        net.close()
    r.close()
    out = dict(seconds=round(sec, 3), increments=len(hist),
               newton_per_increment=round(newton / len(hist), 3),
               cg_per_increment=round(cg / len(hist), 2))
    if adaptive:
        out.update(substeps=sub, cutbacks=cuts)
    return out, sig


def paper_workloads(stream):
    """The paper's own histories (R = 0 triangles of period 4 s, Eq. 28 as
    intended; 235 grains, discrete operator, tol 1e-6):
    * the performance case of Sec. 5: three cycles at 1 % on 32^3, 64^3 and
      128^3, whole-history wall time of the chosen paths and of plain FP64;
    * three cycles at 5 % on 64^3 with automatic time incrementation,
      mixed against FP64 per cycle (Eq. 29);
    * one hundred cycles at 1 % on 32^3: drift of mixed precision against
      FP64 and of the continuous against the discrete operator, per cycle
      (Eq. 29), and the stable cycle's peak stress."""
    from synthetic import config_by_name
    out = {}
    perf = {}
    for name in ("P1_32", "P1_64", "P1_128"):
        cfg = config_by_name(name)
        micro, hist = cfg.microstructure(), cfg.history()
        row = {}
        # the chosen path (mixed, learned start, inexact-Newton forcing),
        # mixed alone, plain FP64
        for label, prec, learned in (("mixed_learned", "mixed", True),
                                     ("mixed", "mixed", False),
                                     ("fp64", "fp64", False)):
            row[label], _ = _run_history(micro, hist, prec, "discrete", stream,
                                         learned=learned,
                                         forcing=FORCING if learned else 0)
        perf[f"{cfg.n}^3"] = row
        print(f"paper workload {name} done", file=sys.stderr, flush=True)
    out["r0_1pct_3cycles"] = perf
    cfg = config_by_name("P2")
    micro, hist = cfg.microstructure(), cfg.history()
    m, sm = _run_history(micro, hist, "mixed", "discrete", stream, adaptive=True)
    f, sf = _run_history(micro, hist, "fp64", "discrete", stream, adaptive=True)
    out["r0_5pct_3cycles_64"] = dict(
        mixed=m, fp64=f, peak_sigma11=float(np.max(sf)),
        eq29_mixed_vs_fp64_pct_per_cycle=_eq29_per_cycle(sm, sf,
                                                         cfg.inc_per_cycle))
    print("paper workload P2 done", file=sys.stderr, flush=True)
    cfg = config_by_name("P3")
    micro, hist = cfg.microstructure(), cfg.history()
    m, sm = _run_history(micro, hist, "mixed", "discrete", stream)
    f, sf = _run_history(micro, hist, "fp64", "discrete", stream)
    c, sc = _run_history(micro, hist, "fp64", "continuous", stream)
    k = cfg.inc_per_cycle
    dm = _eq29_per_cycle(sm, sf, k)
    dc = _eq29_per_cycle(sc, sf, k)
    peaks = [float(np.max(sf[i:i + k])) for i in range(0, len(sf), k)]
    out["r0_1pct_100cycles_32"] = dict(
        mixed=m, fp64=f, fp64_continuous=c,
        eq29_mixed_vs_fp64_pct=dict(first=dm[0], last=dm[-1], max=max(dm)),
        eq29_continuous_vs_discrete_pct=dict(first=dc[0], last=dc[-1],
                                             max=max(dc)),
        peak_sigma11_cycle=dict(first=peaks[0], second=peaks[1],
                                last=peaks[-1]))
    print("paper workload P3 done", file=sys.stderr, flush=True)
    return out


def paper_case(stream):
    """The performance case of the paper (Sec. 5): three R = 0 cycles at
    1 % (Eq. 28 as intended, 40 increments per cycle) on a 32^3 RVE of 235
    grains, discrete operator, tol 1e-6; whole-history wall time of the
    chosen path (mixed, learned start, forcing) and of plain FP64, and
    their macroscopic loops against each other (Eq. 29)."""
    from synthetic import config_by_name
    cfg = config_by_name("P1_32")
    micro, hist = cfg.microstructure(), cfg.history()
    ch, s_ch = _run_history(micro, hist, "mixed", "discrete", stream,
                            learned=True, forcing=FORCING)
    fp, s_fp = _run_history(micro, hist, "fp64", "discrete", stream)
    s_ch, s_fp = np.array(s_ch), np.array(s_fp)
    return {"workload": (f"{cfg.n}^3 RVE, {cfg.grains} grains, 3 R = 0 cycles "
                         f"at 1 %, 40 increments per cycle, tol 1e-6"),
            "chosen": ch, "fp64": fp,
            "chosen_over_fp64": round(fp["seconds"] / ch["seconds"], 3),
            "eq29_chosen_vs_fp64": float(np.max(np.abs(s_ch - s_fp))
                                         / np.max(np.abs(s_fp)))}


def predictor_stats(infos):
    return dict(
        newton_per_increment=float(np.mean([i["newton_iters"] for i in infos])),
        cg_per_increment=float(np.mean([i["cg_iters_total"] for i in infos])),
        median_predictor_residual=float(np.median(
            [i["predictor_residual"] for i in infos])),
        learned_start_used=float(np.mean([i["used_learned"] for i in infos])),
        learned_kept_directly=float(np.mean(
            [i["plain_predictor_residual"] < 0 for i in infos])))


def oracle_sample(micro, hist, gpu_infos, budget_s):
    """Time the CPU oracle on a bounded sample of the same workload.

    The sample is the first increment's building blocks at full size: one
    constitutive evaluation (with tangent), one FP64 residual G(P) and CG
    matvecs G(K:p), timed on this host.  Scaled by the GPU run's average
    counts per increment (evaluations = Newton corrections + 1, residuals
    likewise, matvecs = CG iterations) it estimates the oracle's seconds
    per increment.
    """
    from oracle.solver import OracleRVE
    from synthetic import material_params
    o = OracleRVE((micro.n,) * 3, micro.phase, micro.quat, micro.law,
                  material_params(), "discrete")
    inc = hist[0]
    F = o.F + (inc["F_bar"] - o.F_bar)[None]
    t0 = time.perf_counter()
    P, K, _, _ = o.constitutive(F, inc["dt"], np.zeros((o.N, 12)))
    t_const = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = o.G(P)
    t_res = time.perf_counter() - t0
    Kv = K.reshape(o.N, 9, 9)
    reps = 0
    t0 = time.perf_counter()
    x = r.copy()
    while True:
        y = np.einsum("vab,vb->va", Kv, x.reshape(o.N, 9))
        x = o.G(y.reshape(o.N, 3, 3))
        reps += 1
        if time.perf_counter() - t0 > max(0.0, budget_s - t_const - t_res) \
                or reps >= 8:
            break
    t_mv = (time.perf_counter() - t0) / reps
    newton = np.mean([i["newton_iters"] for i in gpu_infos])
    cgit = np.mean([i["cg_iters_total"] for i in gpu_infos])
    sec_per_inc = (newton + 1) * (t_const + t_res) + cgit * t_mv
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f
                       if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return dict(value=o.N / sec_per_inc, unit="voxel-increments/s",
                cores=len(os.sched_getaffinity(0)), kind="oracle", cpu=cpu,
                sample=(f"64^3 increment 1 building blocks on this host: "
                        f"1 constitutive eval {t_const:.2f}s, 1 FP64 residual "
                        f"{t_res:.2f}s, {reps} CG matvecs {t_mv:.2f}s each; "
                        f"scaled by the GPU run's mean {newton + 1:.2f} "
                        f"evaluations and {cgit:.1f} CG iterations per "
                        f"increment"),
                seconds_per_increment=sec_per_inc)


# ----------------------------------------------------------------- oracle leg
# Everything below up to PMC_SUMMARY calls the CPU oracle: the end-to-end
# oracle timing of the 16^3 history and the error checks of the GPU results
# against the oracle.  It runs only in the cpu_baseline leg (not with
# --no-cpu), after the timed GPU legs or in a separate process on its own
# cores while they run.

def _oracle_point_law_chunk(args):
    """The oracle's point law at given F from a committed state (crystal
    grains and SVK particles): returns (P, slips, ok)."""
    from oracle import crystal, material
    from synthetic import material_params
    F, Fpi0, chi0, label, quat, law, dt = args
    p = material_params()
    S0g, Cg = crystal.grain_tables(quat, p)
    lam, mu = crystal.lame_from_young(p[8], p[9])
    n = F.shape[0]
    P = np.zeros((n, 3, 3))
    dg = np.zeros((n, 12))
    ok = np.ones(n, dtype=bool)
    cp = np.nonzero(law[label] == 0)[0]
    el = np.nonzero(law[label] == 1)[0]
    if cp.size:
        g = label[cp]
        out = material.cp_update(F[cp], Fpi0[cp], chi0[cp],
                                 np.zeros((cp.size, 12)), S0g[g], Cg[g], p,
                                 dt, tangent=False)
        P[cp], dg[cp], ok[cp] = out["P"], out["dg"], out["ok"]
    if el.size:
        P[el] = material.svk_update(F[el], lam, mu, False)["P"]
    return P, dg, ok


def oracle_errors(chk, micro, operator, pool, max_voxels=None, residual=True):
    """Errors of a GPU-solved increment against the oracle: the equilibrium
    residual ||G(P)|| / ||P|| with the oracle's G (Eq. 11), the point law
    re-integrated by the oracle from the committed state at the GPU's F
    (every voxel, or a seeded sample of max_voxels), and <F> - F_bar."""
    from oracle.solver import OracleRVE
    from synthetic import material_params
    N = micro.n ** 3
    F = chk["F"].T.reshape(N, 3, 3)
    P = chk["P"].T.reshape(N, 3, 3)
    Fpi0 = chk["Fpi0"].T.reshape(N, 3, 3)
    chi0 = chk["chi0"].T
    dg = chk["dg"].T
    out = {"increment": chk["k"], "gpu_residual_rel": chk["residual_rel"]}
    if residual:
        o = OracleRVE((micro.n,) * 3, micro.phase, micro.quat, micro.law,
                      material_params(), operator)
        out["residual_rel_oracle_G"] = float(np.linalg.norm(o.G(P))
                                             / np.linalg.norm(P))
        fl = F - chk["F_bar"].reshape(1, 3, 3)
        out["incompatibility_rel_oracle_G"] = float(
            np.linalg.norm(o.G(fl) - fl) / np.linalg.norm(fl))
    idx = np.arange(N)
    if max_voxels is not None and max_voxels < N:
        idx = np.sort(np.random.default_rng(11).choice(N, max_voxels,
                                                       replace=False))
    chunks = np.array_split(idx, max(1, min(len(idx) // 8192, 64)))
    res = list(pool.map(_oracle_point_law_chunk, [
        (F[c], Fpi0[c], chi0[c], micro.phase[c], micro.quat, micro.law,
         chk["dt"]) for c in chunks]))
    Pref = np.concatenate([x[0] for x in res])
    dgref = np.concatenate([x[1] for x in res])
    out["point_law_voxels"] = int(len(idx))
    out["point_law_local_failures"] = int(sum((~x[2]).sum() for x in res))
    out["point_law_P_max_rel"] = float(np.max(np.abs(P[idx] - Pref))
                                       / np.max(np.abs(Pref)))
    out["point_law_slip_max_rel"] = float(np.max(np.abs(dg[idx] - dgref))
                                          / max(np.max(np.abs(dgref)), 1e-300))
    out["mean_F_minus_F_bar_max"] = float(np.max(np.abs(
        F.mean(axis=0) - chk["F_bar"].reshape(3, 3))))
    return out


def _c1_oracle_history(q, cores):
    """Child process: the oracle solves the 16^3 history end to end (20
    increments, tol 1e-6, CG 1e-4, the tolerances of the GPU paths)."""
    try:
        os.sched_setaffinity(0, cores)
    except (AttributeError, OSError):
        pass
    from oracle.solver import OracleRVE
    from synthetic import config_by_name, material_params
    cfg = config_by_name("C1")
    micro = cfg.microstructure()
    hist = cfg.history()
    o = OracleRVE((micro.n,) * 3, micro.phase, micro.quat, micro.law,
                  material_params(), cfg.operator)
    sig, newton, cg = [], 0, 0
    t0 = time.perf_counter()
    for inc in hist:
        if inc["cycle_start"]:
            o.reset_fips()
        info = o.increment(inc["F_bar"], inc["dt"], tol=1e-6, eta=1e-4)
        if info.status != 0:
            q.put(dict(error=f"oracle increment {inc['k']}: {info.status}"))
            return
        sig.append(float(info.sigma_bar[0, 0]))
        newton += info.newton_iters
        cg += info.cg_iters_total
    sec = time.perf_counter() - t0
    q.put(dict(seconds=sec, increments=len(hist), voxels=micro.n ** 3,
               newton=newton, cg=cg, sigma11=sig, cores=len(cores)))


class OracleLeg:
    """The CPU oracle beside the GPU run: the 16^3 history timed end to end
    in a child process pinned to half of this process's cores (started
    before the GPU legs, which keep the other half), then error checks of
    the GPU results after the timed legs."""

    def __init__(self):
        import multiprocessing as mp
        cores = sorted(os.sched_getaffinity(0))
        half = max(1, len(cores) // 2)
        self.gpu_cores = set(cores[:half]) if len(cores) > 1 else set(cores)
        self.cpu_cores = set(cores[half:]) if len(cores) > 1 else set(cores)
        self.all_cores = set(cores)
        ctx = mp.get_context("spawn")
        self.q = ctx.Queue()
        saved = {k: os.environ.get(k) for k in THREAD_VARS}
        for k in THREAD_VARS:
            os.environ[k] = str(len(self.cpu_cores))
        self.proc = ctx.Process(target=_c1_oracle_history,
                                args=(self.q, self.cpu_cores), daemon=True)
        self.proc.start()
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
        try:
            os.sched_setaffinity(0, self.gpu_cores)
        except OSError:
            pass

    def c1_result(self, timeout=900):
        import queue
        t0 = time.perf_counter()
        while True:
            try:
                res = self.q.get(timeout=30)
                break
            except queue.Empty:
                waited = time.perf_counter() - t0
                if waited > timeout or not self.proc.is_alive():
                    res = dict(error="the oracle's 16^3 history did not finish")
                    break
                print(f"bench: oracle 16^3 history still running "
                      f"({waited:.0f} s waited)", file=sys.stderr, flush=True)
        self.proc.join(timeout=30)
        try:
            os.sched_setaffinity(0, self.all_cores)
        except OSError:
            pass
        return res

    def pool(self):
        import concurrent.futures as cf
        import multiprocessing as mp
        return cf.ProcessPoolExecutor(
            max_workers=max(1, min(16, len(self.all_cores))),
            mp_context=mp.get_context("spawn"))


THREAD_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def gpu_c1_history(stream):
    """The 16^3 history on the GPU in FP64 with the homogeneous predictor
    (the oracle's method), same tolerances: seconds and sigma_11."""
    import torch
    from synthetic import config_by_name
    cfg = config_by_name("C1")
    micro = cfg.microstructure()
    out, sig = _run_history(micro, cfg.history(), "fp64", cfg.operator, stream)
    return out, sig, micro.n ** 3


PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic_c3_64cubed.json")


def pmc_traffic(kernel, fused=False):
    """HBM bytes per dispatch of a kernel class from the committed
    FETCH_SIZE/WRITE_SIZE runs (scaled by the copy-kernel calibration), or
    None when there is no such measurement, the kernel's source file has
    changed since it was taken, or the CG schedule (K:p folded into pass A
    or not) differs from the measured one."""
    import hashlib
    try:
        with open(PMC_SUMMARY) as f:
            summ = json.load(f)
        k = summ["kernels"][kernel]
        if (kernel.startswith("matvec_")
                and bool(summ.get("fused", False)) != bool(fused)):
            return None
        with open(os.path.join(ROOT, k["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != k["source_sha256"]:
                return None
        return float(k["traffic_bytes_per_dispatch"])
    except (OSError, KeyError, ValueError):
        return None


def live_report(live, rmc, N, cg_total, sample=None, fused=False, seen=None):
    """Per-kernel live durations, FFT bandwidth and the dominant kernel's
    roofline from the event timings of the timed region.  The dominant
    kernel is the one with the largest total time per increment over the
    sample increments in which every hot-path kernel was timed (the CG
    kernels are not timed in the timed region: one event pair per launch
    would cost several per cent of the throughput); its roofline uses the
    timed region's live durations when it is timed there, else the
    sample's."""
    pb = pass_bytes(fused)
    avg_ms = {k: (ms / n if n else None) for k, (ms, n) in live.items()}
    launches = {k: n for k, (ms, n) in live.items()}
    # every launch of a class (the CG classes are timed on a sample of them)
    allk = {k: (seen[k] if seen and seen.get(k) else launches[k]) for k in live}
    # time of all launches: the sampled average times every launch
    total_ms = {k: (avg_ms[k] * allk[k] if avg_ms[k] else 0.0) for k in live}
    # matvec passes: bytes actually streamed = per-voxel bytes x voxels x
    # CG iterations done (launches past convergence in a replayed chunk
    # return at once and move nothing)
    mv = ("matvec_pass_a", "matvec_pass_b", "matvec_pass_c")  # FFT passes
    mv_ms = sum(total_ms[k] for k in mv)
    fft_gbs = (N * cg_total * sum(pb[k] for k in mv)
               / (mv_ms * 1e-3) / 1e9) if all(launches[k] for k in mv) else None
    rm_f64 = (RM_FLOPS["eval64"] * rmc["evals"] + RM_FLOPS["step64"] * rmc["steps"]
              + RM_FLOPS["crystal64"] * rmc["crystal"]
              + RM_FLOPS["particle64"] * rmc["particle"])
    rm_f32 = RM_FLOPS["eval32"] * rmc["evals"] + RM_FLOPS["step32"] * rmc["steps"]
    rm_flops = rm_f64 + rm_f32

    def hbm(k):
        per_launch = N * pb[k] * cg_total / allk[k]
        ach = per_launch / (avg_ms[k] * 1e-3) / 1e9
        return dict(kernel=k, bound="hbm", achieved=round(ach, 1),
                    peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=pmc_traffic(k, fused),
                    bytes_per_launch=round(per_launch), avg_ms=round(avg_ms[k], 5),
                    launches=allk[k], launches_timed=launches[k])

    def alu():
        # FP32 work is charged at the FP64 rate: the library is compiled
        # without the packed FP32 instructions that double the FP32 vector
        # peak
        per_launch = rm_flops / launches["return_map"]
        ach = per_launch / (avg_ms["return_map"] * 1e-3) / 1e12
        return dict(kernel="return_map", bound="alu", achieved=round(ach, 3),
                    peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(ach / FP64_PEAK_TFLOPS, 4),
                    traffic=pmc_traffic("return_map"),
                    flops_per_launch=round(per_launch),
                    flops_fp64_per_launch=round(rm_f64 / launches["return_map"]),
                    flops_fp32_per_launch=round(rm_f32 / launches["return_map"]),
                    avg_ms=round(avg_ms["return_map"], 4),
                    launches=launches["return_map"])

    timed = {k: v for k, v in total_ms.items() if launches[k]}
    dom = max(timed, key=lambda k: timed[k])
    share = None
    if sample is not None:
        st = {k: ms for k, (ms, n) in sample["timing"].items() if n}
        tot = sum(st.values())
        share = {k: round(v / tot, 4) for k, v in
                 sorted(st.items(), key=lambda kv: -kv[1])}
        dom = max(st, key=lambda k: st[k])
    if dom in live_classes(fused) or sample is None:
        roof = (hbm(dom) if dom in pb else
                (alu() if dom == "return_map" else None))
        if roof is not None:
            roof["timed_over"] = (
                "timed region (HIP events on the launch"
                + (f"; one launch in {LIVE_CG_STRIDE} of the CG kernels)"
                   if roof["kernel"].startswith("matvec") else ")"))
    else:
        ms, n = sample["timing"][dom]
        per_launch = N * pb[dom] * sample["cg_total"] / n
        ach = per_launch / (ms / n * 1e-3) / 1e9
        roof = dict(kernel=dom, bound="hbm", achieved=round(ach, 1),
                    peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=pmc_traffic(dom, fused),
                    bytes_per_launch=round(per_launch),
                    avg_ms=round(ms / n, 5), launches=n,
                    timed_over=("increments %d-%d before the timed region, "
                                "every kernel timed (HIP events per launch)"
                                % tuple(sample["increments"])))
    rep = {
        "fft_gbps": round(fft_gbs, 1) if fft_gbs else None,
        "kernel_avg_ms_live": {k: (round(v, 5) if v else v)
                               for k, v in avg_ms.items()},
        "kernel_total_ms_live": {k: round(v, 3) for k, v in total_ms.items()},
        "kernel_launches_live": allk,
        "kernel_launches_timed_live": launches,
        "return_map_work": dict(rmc, flops=rm_flops, flops_fp64=rm_f64,
                                flops_fp32=rm_f32),
        "roofline": roof,
    }
    if share is not None:
        rep["kernel_time_share_sample"] = dict(
            increments=sample["increments"], share=share)
        rep["kernel_avg_ms_sample"] = {
            k: round(ms / n, 5) for k, (ms, n) in sample["timing"].items() if n}
    for k in pb:
        if launches[k] and k != dom:
            rep[k + "_roofline"] = hbm(k)
    if launches["return_map"] and dom != "return_map":
        rep["return_map_roofline"] = alu()
    return rep


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on exactly one GPU; "
                          "multi-GPU runs are not implemented (see the design "
                          "notes for how the path would shard)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    global FORCING, LIVE_CG_STRIDE
    FORCING = args.forcing_mode
    if args.live_cg_stride < 1:
        raise SystemExit("--live-cg-stride must be at least 1")
    LIVE_CG_STRIDE = args.live_cg_stride
    import torch
    from synthetic import config_by_name
    cfg = config_by_name(args.config)
    micro = cfg.microstructure()
    hist = cfg.history()
    if max(args.warmup, args.start or 0) + args.steps > len(hist):
        raise SystemExit(f"the {cfg.name} history has {len(hist)} increments; "
                         f"warmup + steps must not exceed it")
    # the oracle's end-to-end run of the 16^3 history starts first, in a
    # child process on half of the cores (the GPU legs keep the other half)
    oleg = None if args.no_cpu else OracleLeg()
    stream = torch.cuda.Stream()
    calib = copy_calibration(stream) if args.copy_calibration else None
    with torch.cuda.stream(stream):
        chosen = run_path(micro, hist, "mixed", args.graph, args.steps,
                          args.warmup, stream, live=not args.no_live,
                          learned=not args.no_learned, start=args.start,
                          cg_chunk=args.cg_chunk, with_fips=True,
                          forcing=0 if args.no_forcing else FORCING,
                          schedule=(tuple(int(x) for x in
                                          args.fft_schedule.split(","))
                                    if args.fft_schedule else None),
                          check=oleg is not None,
                          sample_all=not args.no_live)
        progress("chosen path done")
        plain = None
        if not args.no_plain:
            plain = run_path(micro, hist, "fp64", False, args.steps,
                             args.warmup, stream, live=False, start=args.start,
                             cg_chunk=args.cg_chunk)
            progress("plain path done")
        ablations = None
        if not args.no_ablations:
            # what each addition of the chosen path contributes: the same
            # window solved with one more addition at a time
            ablations = {}
            for label, prec, ws, frc in (
                    ("fp64_forcing", "fp64", 0, FORCING),
                    ("mixed_forcing", "mixed", 0, FORCING),
                    ("mixed_forcing_extrapolated_start", "mixed", 3, FORCING)):
                ablations[label] = run_path(
                    micro, hist, prec, False, args.steps, args.warmup, stream,
                    live=False, start=args.start, cg_chunk=args.cg_chunk,
                    forcing=frc, warm_start=ws)
                progress(f"ablation {label} done")
    N = micro.n ** 3
    value = N * args.steps / chosen["elapsed"]
    infos = chosen["infos"]
    cg_per_inc = float(np.mean([i["cg_iters_total"] for i in infos]))
    newton_per_inc = float(np.mean([i["newton_iters"] for i in infos]))
    cg_total = sum(i["cg_iters_total"] for i in infos)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "voxel-increments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * chosen["elapsed"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": (f"{cfg.name}: {cfg.n}^3 RVE, {cfg.grains} "
                                f"Voronoi grains + {cfg.particle_fraction:.0%}"
                                f" stiff particles, {cfg.operator} operator, "
                                f"+-{cfg.eps_a:.1%} cycles, "
                                f"{cfg.inc_per_cycle} inc/cycle, tol 1e-6"),
                   "voxels": N, "precision": "mixed FP32 FFT/CG + FP64",
                   "graph": args.graph,
                   "cg_chunk": args.cg_chunk,
                   "cg_forcing": 0 if args.no_forcing else FORCING,
                   "warm_start": ("homogeneous" if args.no_learned else
                                  "learned (weights/warmstart.npy), kept "
                                  "directly below half the homogeneous "
                                  "predictor's last residual, else the "
                                  "better of both"),
                   "timed_increments": [chosen["start"] + 1,
                                        chosen["start"] + args.steps],
                   "timed_window": ("last cycle of the history, held out from "
                                    "the warm-start training"
                                    if (args.start is None and
                                        args.steps <= cfg.inc_per_cycle) else
                                    "increments of the history"),
                   "fft_schedule": chosen["schedule"]},
        "newton_per_increment": newton_per_inc,
        "cg_per_increment": cg_per_inc,
        "predictor": predictor_stats(infos),
        "nonlocal_fips": chosen["nonlocal_"],
        "cg_passes": chosen["passes"],
    }
    live = chosen["live"]
    if live is not None:
        out.update(live_report(live, chosen["rm_counts"], N, cg_total,
                               chosen["sample"],
                               bool(chosen["schedule"]["fused"]),
                               chosen["seen"]))
    if out.get("fft_gbps") is None and chosen["passes"]:
        out["fft_gbps"] = chosen["passes"]["fft_projection_passes"]["gbps"]
    if plain is not None:
        pv = N * args.steps / plain["elapsed"]
        out["plain"] = {"value": round(pv, 1), "unit": "voxel-increments/s",
                        "ms_per_step": round(1e3 * plain["elapsed"] / args.steps, 3),
                        "dtype": "f64",
                        "cg_per_increment": float(np.mean(
                            [i["cg_iters_total"] for i in plain["infos"]])),
                        "newton_per_increment": float(np.mean(
                            [i["newton_iters"] for i in plain["infos"]])),
                        "predictor": predictor_stats(plain["infos"])}
        out["chosen_over_plain"] = round(value / pv, 3)
        s_c = np.array(chosen["sigma11"])
        s_p = np.array(plain["sigma11"])
        out["sigma11_max_rel_diff_vs_plain"] = float(
            np.max(np.abs(s_c - s_p)) / np.max(np.abs(s_p)))
        if ablations is not None:
            rows = {"fp64 (plain)": out["plain"]}
            for label, res in ablations.items():
                v = N * args.steps / res["elapsed"]
                rows[label] = dict(
                    value=round(v, 1),
                    ms_per_step=round(1e3 * res["elapsed"] / args.steps, 3),
                    over_plain=round(v / pv, 3),
                    sigma11_max_rel_diff_vs_plain=float(
                        np.max(np.abs(np.array(res["sigma11"]) - s_p))
                        / np.max(np.abs(s_p))),
                    **predictor_stats(res["infos"]))
            rows["mixed_forcing_learned_start (chosen)"] = dict(
                value=out["value"], ms_per_step=out["ms_per_step"],
                over_plain=out["chosen_over_plain"], **out["predictor"])
            out["ablations"] = {
                "window": out["config"]["timed_increments"],
                "note": ("each row adds one thing to the one before: "
                         "inexact-Newton forcing (mode %d), FP32 FFT/CG, the "
                         "extrapolated start (last fluctuation increment x "
                         "load ratio, kept by the rule of the learned "
                         "start), the learned start" % FORCING),
                "rows": rows}
    if not args.no_batch:
        with torch.cuda.stream(stream):
            out["batch"] = batch_run(args.batch_steps, stream)
        progress("batch done")
    if args.large_steps > 1:
        with torch.cuda.stream(stream):
            out["large_rve"] = large_run(args.large_steps, stream)
        progress("128^3 done")
    if not args.no_umat:
        out["umat_bridge"] = umat_run(stream)
    if not args.no_paper_case:
        with torch.cuda.stream(stream):
            out["paper_case_32"] = paper_case(stream)
        progress("paper case done")
    if args.paper_workloads:
        with torch.cuda.stream(stream):
            out["paper_workloads"] = paper_workloads(stream)
    c1_gpu = None
    if oleg is not None:
        with torch.cuda.stream(stream):
            c1_gpu = gpu_c1_history(stream)
    if calib:
        out["copy_calibration"] = calib
    cbw = copy_bandwidth(stream)
    out["measured_copy_gbps"] = cbw
    if out.get("roofline") and out["roofline"].get("unit") == "GB/s":
        out["roofline"]["frac_of_measured_copy"] = round(
            out["roofline"]["achieved"] / cbw, 4)
    if out.get("cg_passes"):
        out["cg_passes"]["fft_projection_passes"]["frac_of_measured_copy"] = \
            round(out["cg_passes"]["fft_projection_passes"]["gbps"] / cbw, 3)
    batch_chk = out.get("batch", {}).pop("_check", None)
    batch_micro = out.get("batch", {}).pop("_micro0", None)
    large_chk = out.get("large_rve", {}).pop("_check", None)
    large_micro = out.get("large_rve", {}).pop("_micro", None)
    if oleg is not None:
        # the oracle leg: its end-to-end run of the 16^3 history (done in
        # the child meanwhile), error checks of the GPU results, and the
        # bounded sample of the 64^3 workload itself
        progress("waiting for the oracle's 16^3 history")
        c1 = oleg.c1_result()
        progress("oracle 16^3 history done; error checks")
        errs = {}
        with oleg.pool() as pool:
            errs["chosen_64"] = oracle_errors(chosen["check"], micro,
                                              cfg.operator, pool)
            if batch_chk is not None:
                errs["batch_rve0"] = oracle_errors(batch_chk, batch_micro,
                                                   "discrete", pool)
                errs["batch_rve0"]["edge"] = batch_micro.n
            if large_chk is not None:
                errs["large_128"] = oracle_errors(
                    large_chk, large_micro, "discrete", pool,
                    max_voxels=131072, residual=False)
                errs["large_128"]["note"] = (
                    "point law on a seeded sample of voxels; the dense-DFT "
                    "oracle G at 128^3 takes minutes and is compared "
                    "element-wise in the tests instead")
        out["error_vs_oracle"] = errs
        progress("error checks done; oracle sample of the 64^3 workload")
        # the oracle implements the homogeneous-predictor method: scale its
        # sample by the plain path's counts when they are there
        ref = plain["infos"] if plain is not None else infos
        cb = oracle_sample(micro, hist, ref, args.cpu_seconds)
        if "error" not in c1 and c1_gpu is not None:
            g_out, g_sig, n1 = c1_gpu
            vo = n1 * c1["increments"] / c1["seconds"]
            vg = n1 * g_out["increments"] / g_out["seconds"]
            sg, so = np.array(g_sig), np.array(c1["sigma11"])
            cb["end_to_end_16"] = dict(
                workload=("16^3 RVE, 8 grains, continuous operator, 20 "
                          "increments of a +-1 % cycle, tol 1e-6, homogeneous "
                          "predictor, FP64, solved end to end"),
                oracle_seconds=round(c1["seconds"], 2),
                oracle_value=round(vo, 1), oracle_cores=c1["cores"],
                gpu_fp64_seconds=g_out["seconds"], gpu_fp64_value=round(vg, 1),
                gpu_over_oracle=round(vg / vo, 1),
                eq29_gpu_vs_oracle=float(np.max(np.abs(sg - so))
                                         / np.max(np.abs(so))))
        elif "error" in c1:
            cb["end_to_end_16"] = c1
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
