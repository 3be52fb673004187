"""Benchmark: ML-CG ptychography on one MI355X.

Workload: the single large projection -- 2048^2 complex64 object, 128^2
apodised-disk probe, 64x64 = 4096 positions on a 24 px raster with +-2 px
jitter, 128^2 float32 Poisson intensities at 1e5 photons per pattern,
object-only CG with FP64 reductions.  Inputs come from the seeded generator
(object, probe, scan; Poisson counts drawn on the host from the generator's
per-chunk seeds) with the expected intensities from a float64 host forward
model of the complex64 object and probe: the data are the tested workload's.
A step is one CG iteration (GRAD -> DIR -> LS -> Update over all 4096
patterns).  W warm-up iterations run in a separate solve; the
timed region is one ptyg_cg_solve of K iterations from the usual start
(psi_0 = 1), inputs resident in HBM.

value = diffraction patterns per second through grad + line search
(4096 * K / t).  The roofline object is the forward+adjoint unit, the GRAD
stage as the solver runs it (transform kernel, ordered overlap sum and
reductions), at its algorithmic 20 bytes per pattern pixel, its duration
measured by HIP events on the launch stream inside the timed region; the
per-kernel fractions follow as secondary fields.  The CPU baseline is the
FP64 oracle on a bounded sample of the same workload.  `warm_start` (c2)
holds the metric's second half: wall time for the learned warm start
(inference, stitch, CG to plain CG's final objective) against plain CG's
100 iterations, with iteration counts and errors against the truth.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic bytes per launch (what each kernel must move; overlapping patch
# re-reads served by caches still count), P = K n^2 pattern pixels:
#   GRAD: patch 8 B + intensity 4 B + per-pattern back-propagated wave 8 B
#         per pixel (+ 8 B stored G psi in the batched search)
#   sequential line-search trial: psi and eta patches 16 B + intensity 4 B
#   batched line-search pass: per listed (d > 0) element index 4 B + A 8 B +
#         B 8 B + intensity 4 B
#   direction forward: eta patch 8 B + far field 8 B + stored A read 8 B
#   overlap sum: back-propagated waves 8 B per pixel + object gradient write
def kernel_bytes(kind: str, cfg, batched: bool, nnz: int, joint: bool = False) -> int:
    """Algorithmic bytes per launch.  GRAD kernel and GRAD stage: 20 B per
    pattern pixel (patch 8, intensity 4, gradient contribution 8); the far
    field the batched search stores is not counted.  Line-search pass,
    direction forward and overlap sum as commented above."""
    px = cfg.k * cfg.n * cfg.n
    compact = batched and not joint and cfg.n == 128
    stored = 8 * nnz + px // 4 if compact else 8 * px
    if kind in ("grad", "grad_unit"):
        return 20 * px
    if kind == "minfunc":
        if not batched:
            return 20 * px
        # A, B (and C) and d per listed element, plus its index unless compacted
        return (20 if compact else 24 + (8 if joint else 0)) * nnz
    if kind == "dir_forward":
        if joint:
            # (psi and eta patches, b stored) then (eta patch, c stored)
            return 40 * px
        return 8 * px + stored
    if kind == "tile_sum":
        return 8 * px + 8 * cfg.obj_h * cfg.obj_w
    raise KeyError(kind)


KERNEL_NAMES = {"grad": "k_grad (fused GRAD)", "minfunc": "k_minfunc (line-search trial)",
                "ls_batched": "k_ls_batch (batched line-search pass)", "dir_forward": "k_fwd_t (G eta)",
                "tile_sum": "k_tile_sum (ordered overlap sum)",
                "grad_unit": "GRAD stage: k_grad + k_tile_sum + k_finalize (forward+adjoint unit)"}
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch (FETCH_SIZE x 2 + WRITE_SIZE x 1, the factors from a
# 512 MiB device copy measured by the same counters) of the current kernels,
# from the rocprofv3 --pmc runs summarised in profiles/; keyed (kind,
# workload, line search); absent = not measured for the current kernel build
TRAFFIC_BYTES = {
    # solver GRAD kernel 1078.9 MB + ordered overlap sum 710.7 MB (+ finalize < 1 MB),
    # profiles/cg_c2_batched_ls_hbm_bytes.md
    ("grad_unit", "c2", "batched"): 1744.6e6,
}
FP32_PEAK_TFLOPS = 157.3


def fft_flops(n: int) -> float:
    m = n * n
    return 5.0 * m * math.log2(m)


def warm_start(args, inp, probe, pos, data, device) -> dict:
    """Second half of the metric: time to plain CG's final objective from
    the learned warm start against plain CG from psi_0 = 1, on this run's
    inputs.  The network is trained here (seeded: 500 synthetic 1024^2
    objects, 200 k forward-model patterns, `--warm-start-epochs` epochs,
    then 400 fine-tuning steps through the differentiable operator); the
    timed comparison is warmstart.time_to_objective (plain CG for 100
    iterations; inference on the patterns at least 40 px apart + stitch + CG
    until plain CG's final objective; host wall times around synchronised
    GPU work).  Errors are phase-aligned relative errors against the ground
    truth on the illuminated region."""
    import numpy as np
    import torch

    from paper_2106_07575_amd import warmstart as W

    t0 = time.perf_counter()
    ts = W.make_training_set(probe)
    net = W.Net(device)
    hist = W.train(net, ts, epochs=args.warm_start_epochs)
    del ts
    ft = W.finetune(net, W.finetune_objects(probe), probe, steps=400, lr=3e-4)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    obj_true = torch.from_numpy(inp.obj_true.astype(np.complex64)).to(device)
    r = W.time_to_objective(net, probe, pos, data, tuple(obj_true.shape), obj_true, line_search=args.line_search,
                            infer_sep=40)
    ms = lambda s: round(s * 1e3, 2)
    return {"t_plain_ms": ms(r["t_plain_s"]), "plain_iters": r["plain_iters"],
            "t_warm_ms": ms(r["t_warm_total_s"]), "t_infer_ms": ms(r["t_infer_s"]), "t_stitch_ms": ms(r["t_stitch_s"]),
            "t_cg_warm_ms": ms(r["t_cg_warm_s"]), "warm_iters": r["warm_iters"],
            "warm_reached_target": r["warm_reached_target"], "warm_faster": r["warm_faster"],
            "phi_target": r["phi_plain_final"], "phi_warm_final": r["phi_warm_final"],
            "phi0_ones": r["phi0_ones"], "phi0_warm": r["phi0_warm"],
            "err_plain": round(r["err_plain"], 5), "err_warm": round(r["err_warm"], 5),
            "err_psi0_warm": round(r["err_psi0_warm"], 5), "break_even_iters": round(r["break_even_iters"], 1),
            "inferred_patterns": r["infer_patterns"], "train_epochs": args.warm_start_epochs,
            "train_loss_last": round(float(np.mean(hist[-5:])), 5), "finetune_phi_first_last": [ft[0], ft[-1]],
            "t_train_and_finetune_s": round(t_prep, 1)}


def expected_intensities(obj, probe, pos, chunk: int = 256):
    """|F (p * psi[s_k])|^2 in float64 on the host (Eq. fwd_model with the
    unitary 2-D DFT, scipy's), for input generation only: the counts then
    follow from the same expected values as the tests' workloads."""
    import numpy as np
    import scipy.fft

    n = probe.shape[0]
    out = np.empty((len(pos), n, n))
    for lo in range(0, len(pos), chunk):
        ex = np.stack([probe * obj[r:r + n, c:c + n] for r, c in pos[lo:lo + chunk]])
        out[lo:lo + chunk] = np.abs(scipy.fft.fft2(ex, norm="ortho", workers=-1)) ** 2
    return out


def make_inputs(cfg_name: str, device):
    """Seeded inputs: object, probe and scan from the generator; expected
    intensities |G psi_true|^2 in float64 on the host from the complex64
    object and probe; Poisson counts from the generator's per-chunk seeds."""
    import numpy as np
    import torch

    from paper_2106_07575_amd import synth

    cfg = synth.CONFIGS[cfg_name]
    inp = synth.make_inputs(cfg)
    obj32 = inp.obj_true.astype(np.complex64)
    probe32 = inp.probe.astype(np.complex64)
    inten = expected_intensities(obj32.astype(np.complex128), probe32.astype(np.complex128), inp.pos)
    data = synth.make_data(cfg, inten).astype(np.float32)
    del inten
    probe = torch.from_numpy(probe32).to(device)
    pos = torch.from_numpy(inp.pos).to(device)
    return cfg, inp, probe, pos, torch.from_numpy(data).to(device)


def cpu_baseline(cfg_name: str, halvings_per_iter: float, budget_s: float = 12.0):
    """FP64 oracle on a bounded sample: one GRAD pass plus the mean number of
    line-search passes over the first 512 patterns of the workload (full
    object), repeated until ~budget_s; reported in patterns/s of CG."""
    import numpy as np

    from oracle import ptycho as O
    from paper_2106_07575_amd import synth

    cfg = synth.CONFIGS[cfg_name]
    inp = synth.make_inputs(cfg)
    ks = 512
    pos = inp.pos[:ks]
    probe = inp.probe.astype(np.complex64).astype(np.complex128)
    truth = inp.obj_true.astype(np.complex64).astype(np.complex128)
    data = synth.poisson_counts(np.abs(O.forward(truth, probe, pos)) ** 2, cfg.seed("poisson")).astype(np.float64)
    psi = np.ones(truth.shape, np.complex128)
    eta = np.full(truth.shape, 1e-3 + 0j)
    ntrials = max(1, int(round(halvings_per_iter)))
    t0 = time.perf_counter()
    reps = 0
    while True:
        O.grad(psi, probe, pos, data)
        for j in range(ntrials):
            O.minfunc(psi + 0.5 ** (j + 1) * eta, probe, pos, data)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    per_iter = dt / reps
    return {"value": ks / per_iter, "unit": "patterns/s", "cores": os.cpu_count(), "kind": "oracle",
            "sample": f"{ks} of {cfg.k} patterns of the same workload (full 2048^2 object), 1 GRAD + "
                      f"{ntrials} line-search passes per iteration, {reps} repetitions in {dt:.1f} s, "
                      f"float64, scipy.fft with {os.cpu_count()} workers"}


def run_views(args, device):
    """Multi-view batch: V projections of the 320^2 object / 128^2 probe /
    7x7-position shape (each too small to fill the GPU), one shared probe."""
    import numpy as np
    import torch

    from paper_2106_07575_amd import ptyg, synth

    V = args.views
    objs, poss, datas, probe = [], [], [], None
    for v in range(V):
        cfg = synth.small_config(f"view{v}", 320, 128, 7, 24, 2, photons=1e5, cid=100 + v, iters=args.steps)
        inp = synth.make_inputs(cfg)
        if probe is None:
            probe = torch.from_numpy(inp.probe.astype(np.complex64)).to(device)
        truth = torch.from_numpy(inp.obj_true.astype(np.complex64)).to(device)
        pos = torch.from_numpy(inp.pos).to(device)
        far = ptyg.forward(truth, probe, pos)
        gen = torch.Generator(device=device)
        gen.manual_seed(cfg.seed("poisson"))
        datas.append(torch.poisson((far.real ** 2 + far.imag ** 2).float(), generator=gen))
        poss.append(pos)
    pos = torch.stack(poss)
    data = torch.stack(datas).contiguous()
    k = data.shape[1]
    obj0 = torch.ones((V, 320, 320), dtype=torch.complex64, device=device)
    ls = args.line_search
    ptyg.cg_solve_views(obj0, probe, pos, data, max(1, args.warmup), line_search=ls)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, traces, done = ptyg.cg_solve_views(obj0, probe, pos, data, args.steps, line_search=ls)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ws = ptyg.workspace(ptyg.dims_of((320, 320), 128, k), device, line_search=ls)
    ptyg.cg_solve(obj0[0], probe, pos[0], data[0], max(1, args.warmup), ws=ws, line_search=ls)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v in range(V):
        ptyg.cg_solve(obj0[v], probe, pos[v], data[v], args.steps, ws=ws, line_search=ls)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    print(json.dumps({
        "metric": "diffraction patterns/s through grad+line search (multi-view batch)",
        "value": round(V * k * args.steps / t_batch, 1), "unit": "patterns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_batch / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32 transforms, fp64 reductions", "data": "synthetic",
        "config": {"workload": f"{V} views: 320x320 object, 128x128 probe, {k} positions each, Poisson 1e5",
                   "line_search": ls},
        "one_at_a_time_patterns_per_s": round(V * k * args.steps / t_seq, 1),
        "batch_speedup": round(t_seq / t_batch, 3),
        "final_phi_view0": traces[0][-1]["phi"] if traces and traces[0] else None,
    }))


def run_gd(args, cfg, probe, pos, data, obj0, joint):
    """Gradient descent (Eq. update2) timed like the CG run; CG's objective
    after the same number of iterations (untimed) shows the convergence gap."""
    import torch

    from paper_2106_07575_amd import ptyg

    K = cfg.k
    gamma = args.gd_gamma
    if gamma <= 0.0:
        pa = probe.abs().to(torch.complex64)
        illum, _ = ptyg.adjoint(ptyg.forward(torch.ones_like(obj0), pa, pos), pa, pos, tuple(obj0.shape))
        gamma = 0.1 / float(illum.real.max())
        del illum
    ws = ptyg.workspace(ptyg.dims_of(obj0.shape, cfg.n, K), obj0.device, update_probe=joint)
    est = args.estimator
    if args.warmup > 0:
        ptyg.gd_solve(obj0, probe, pos, data, args.warmup, gamma, update_probe=joint, ws=ws, estimator=est)
    torch.cuda.synchronize()
    ptyg.timing_reset()
    ptyg.timing_enable(True)
    t0 = time.perf_counter()
    _, _, phis = ptyg.gd_solve(obj0, probe, pos, data, args.steps, gamma, update_probe=joint, ws=ws, estimator=est)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ptyg.timing_enable(False)
    kt = ptyg.timing_read()
    wsc = ptyg.workspace(ptyg.dims_of(obj0.shape, cfg.n, K), obj0.device, update_probe=joint, line_search="batched")
    cg = ptyg.cg_solve(obj0, probe, pos, data, args.steps, update_probe=joint, ws=wsc, line_search="batched",
                       estimator=est)
    kinds = {k: {"launches": c, "avg_us": round(ms / c * 1e3, 2)} for k, (ms, c) in kt.items() if c}
    g = kt["grad"]
    avg_s = g[0] / g[1] / 1e3
    alg = kernel_bytes("grad", cfg, False, 0)
    print(json.dumps({
        "metric": "diffraction patterns/s through grad (gradient descent, constant step)",
        "value": round(K * args.steps / dt, 1), "unit": "patterns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32 transforms, fp64 reductions", "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg.obj_h}x{cfg.obj_w} object, {cfg.n}x{cfg.n} probe, {K} "
                               f"positions, Poisson at {cfg.photons:g} photons, gradient descent gamma {gamma:.4g}",
                   "estimator": est},
        "phi_first": phis[0], "phi_last": phis[-1],
        "cg_phi_after_same_iterations": cg.trace[-1]["phi"] if cg.trace else None,
        "kernels": kinds,
        "roofline": {"bound": "hbm", "achieved": round(alg / avg_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / avg_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": KERNEL_NAMES["grad"], "bytes_per_launch": alg, "avg_launch_us": round(avg_s * 1e6, 2)},
    }))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed CG iterations")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2",
                    help="c2 (default: 2048^2, 128^2 probe, object-only) or c5 (8192^2, 256^2 probe, joint "
                         "object+probe from |p|)")
    ap.add_argument("--line-search", default="batched", choices=["batched", "sequential"],
                    help="batched: trials from stored far fields, up to 16 per streaming pass (default); "
                         "sequential: one forward pass per trial")
    ap.add_argument("--estimator", default="ml", choices=["ml", "ls"],
                    help="ml: Poisson maximum likelihood (Eq. ML, the headline); ls: least squares on amplitudes")
    ap.add_argument("--solver", default="cg", choices=["cg", "gd"],
                    help="cg: ML-CG (the headline); gd: gradient descent with a constant step (Eq. update2), "
                         "reported with the objective CG reaches in the same number of iterations")
    ap.add_argument("--gd-gamma", type=float, default=0.0,
                    help="GD step (default 0.1 / peak illumination)")
    ap.add_argument("--views", type=int, default=0,
                    help="multi-view batch: V independent 320^2 / 128^2 / 49-position projections solved in one set "
                         "of launches, against the same V solved one after another")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--warm-start-epochs", type=float, default=2.0,
                    help="c2 only: train the warm-start network this many epochs on forward-model patterns "
                         "(200 k), fine-tune it through the operator, and time NN start + CG to plain CG's final "
                         "objective against plain CG (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the timed run, copy a MIB-MiB device buffer 3 times (a reference kernel of known "
                         "traffic for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the ML-CG hot path here is single-GPU "
              "(multi-GPU sharding is design-only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2106_07575_amd import ptyg

    device = torch.device("cuda:0")
    torch.cuda.set_device(device)
    if args.views > 0:
        run_views(args, device)
        return
    cfg, inp, probe, pos, data = make_inputs(args.config, device)
    K = cfg.k
    joint = args.config == "c5"
    if joint:
        probe = probe.abs().to(torch.complex64)   # amplitude known, phase unknown
    obj0 = torch.ones((cfg.obj_h, cfg.obj_w), dtype=torch.complex64, device=device)
    if args.solver == "gd":
        run_gd(args, cfg, probe, pos, data, obj0, joint)
        return
    ls = args.line_search
    est = args.estimator
    px = K * cfg.n * cfg.n
    batched = ls == "batched"
    # the batched search stores far fields for the pixels with counts only:
    # size its workspace by their number
    nnz = ptyg.listed_count(data, cfg.n)
    max_listed = nnz if batched else -1
    ws = ptyg.workspace(ptyg.dims_of(obj0.shape, cfg.n, K), device, update_probe=joint, line_search=ls,
                        max_listed=max_listed)
    ws_full = ptyg.workspace_size(ptyg.dims_of(obj0.shape, cfg.n, K), update_probe=joint, line_search=ls)

    def kernel_table(kt):
        kinds = {}
        for kind, (ms, cnt) in kt.items():
            if cnt:
                name = "ls_batched" if (kind == "minfunc" and batched) else kind
                avg_s = ms / cnt / 1e3
                ffts = {"grad": 2, "minfunc": 1, "dir_forward": 1 + int(joint), "ls_batched": 0, "tile_sum": 0,
                        "grad_unit": 2}[name]
                kb = kernel_bytes(kind, cfg, batched, nnz, joint)
                kinds[name] = {"kind": kind, "launches": cnt, "avg_us": avg_s * 1e6, "total_ms": ms,
                               "bytes_per_launch": kb, "alg_GBs": kb / avg_s / 1e9,
                               "fft_TFLOPs": ffts * K * fft_flops(cfg.n) / avg_s / 1e12}
        return kinds

    # The timed run records events around the GRAD stage only (the
    # forward+adjoint unit the roofline is about; an event pair adds a few
    # microseconds between launches); a short pass after it, every kind
    # timed, gives the per-kernel table.
    ptyg.timing_reset()
    if args.warmup > 0:
        ptyg.cg_solve(obj0, probe, pos, data, args.warmup, update_probe=joint, ws=ws, line_search=ls, estimator=est,
                      max_listed=max_listed)
    torch.cuda.synchronize()
    ptyg.timing_enable(True, kinds=("grad_unit",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ptyg.cg_solve(obj0, probe, pos, data, args.steps, update_probe=joint, ws=ws, line_search=ls,
                        estimator=est, max_listed=max_listed)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ptyg.timing_enable(False)
    timed = kernel_table(ptyg.timing_read())
    ptyg.timing_reset()
    ptyg.timing_enable(True)
    table_iters = min(args.steps, 10)
    ptyg.cg_solve(obj0, probe, pos, data, table_iters, update_probe=joint, ws=ws, line_search=ls, estimator=est,
                  max_listed=max_listed)
    torch.cuda.synchronize()
    ptyg.timing_enable(False)
    kinds = kernel_table(ptyg.timing_read())

    # the forward+adjoint unit as an API call: K / t(ptyg_grad), one call =
    # tile lists, GRAD, overlap sum and the reductions (events on the stream
    # the binding launches on)
    gws = ptyg.workspace(ptyg.dims_of(obj0.shape, cfg.n, K), device, update_probe=joint)
    for _ in range(3):
        ptyg.grad(res.obj, probe, pos, data, want_probe=joint, ws=gws, estimator=est)
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ncall = 20
    g0.record()
    for _ in range(ncall):
        ptyg.grad(res.obj, probe, pos, data, want_probe=joint, ws=gws, estimator=est)
    g1.record()
    torch.cuda.synchronize()
    grad_call_s = g0.elapsed_time(g1) / ncall / 1e3
    del gws

    iters = res.iters_done
    halvings = sum(r["halvings"] for r in res.trace)
    value = K * iters / dt
    dom = "grad_unit"
    d = timed[dom]
    bpl = d["bytes_per_launch"]
    roofline = {"bound": "hbm", "achieved": round(d["alg_GBs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(d["alg_GBs"] / HBM_PEAK_GBS, 4), "traffic": TRAFFIC_BYTES.get((dom, args.config, ls)),
                "kernel": KERNEL_NAMES[dom], "bytes_per_launch": bpl, "avg_launch_us": round(d["avg_us"], 2),
                "launches": d["launches"], "fft_tflops": round(d["fft_TFLOPs"], 2), "fft_frac_of_fp32_peak":
                    round(d["fft_TFLOPs"] / FP32_PEAK_TFLOPS, 4),
                "per_kernel_frac": {k: round(v["alg_GBs"] / HBM_PEAK_GBS, 4) for k, v in kinds.items()
                                    if k != "grad_unit"}}
    out = {
        "metric": "diffraction patterns/s through grad+line search",
        "value": round(value, 1),
        "unit": "patterns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / max(iters, 1) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 transforms, fp64 reductions",
        "data": "synthetic",
        "config": {"line_search": ls, "estimator": est,
                   "workload": f"{args.config}: {cfg.obj_h}x{cfg.obj_w} complex64 object, {cfg.n}x{cfg.n} probe, "
                               f"{K} positions ({cfg.grid[0]}x{cfg.grid[1]} raster, step {cfg.step}, "
                               f"+-{cfg.jitter} px), Poisson at {cfg.photons:g} photons, "
                               + ("joint object+probe ML-CG" if joint else "object-only ML-CG"),
                   "iterations": iters, "patterns": K},
        "cg_iters_per_s": round(iters / dt, 3),
        # K / t(ptyg_grad) (the call) and K / t(k_grad) (the fused kernel alone)
        "grad_patterns_per_s": round(K / grad_call_s, 1),
        "ptyg_grad_us": round(grad_call_s * 1e6, 1),
        "k_grad_patterns_per_s": (round(K / (timed.get("grad", kinds.get("grad"))["avg_us"] * 1e-6), 1)
                                  if ("grad" in timed or "grad" in kinds) else None),
        "pattern_passes_per_s": round(K * (iters + halvings) / dt, 1),
        "mean_halvings": round(halvings / max(iters, 1), 3),
        "listed_fraction": round(nnz / px, 4),
        "workspace_bytes": int(ws.numel()), "workspace_bytes_all_pixels_reserved": int(ws_full),
        "phi_0": res.trace[0]["phi"] if res.trace else None,
        "final_phi": res.trace[-1]["phi"] if res.trace else None,
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items() if kk != "kind"}
                    for k, v in kinds.items()},
        "kernels_from": f"{table_iters} iterations after the timed run, every kind timed",
        "roofline": roofline,
    }
    if args.copy_calibration:
        src = torch.empty(args.copy_calibration << 20, dtype=torch.uint8, device=device).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel()
    if args.warm_start_epochs > 0 and args.config == "c2" and est == "ml":
        del ws
        out["warm_start"] = warm_start(args, inp, probe, pos, data, device)
    if not args.no_cpu_baseline and not joint and est == "ml":
        out["cpu_baseline"] = cpu_baseline(args.config, halvings / max(iters, 1))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
