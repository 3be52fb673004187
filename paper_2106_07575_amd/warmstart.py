"""Learned CG warm start: a convolutional encoder-decoder predicts, from each
diffraction pattern, the object patch under the probe; the predictions are
phase-synchronised and averaged into the starting guess of ML-CG.

The paper's solver starts CG from a fixed guess (Algorithm 1 takes the
initial object as an input); this module only changes that input.  Plain CG
from psi_0 = 1 stays the fallback and the judge: the warm start is worth it
only if inference + stitching + CG reach plain CG's final objective in less
wall time.

Network (NHWC, BF16 operands on MFMA, FP32 accumulation, all layers in
libptyg.so): input 0.1 log(1 + d), 128^2 x 1 -> 4 levels (32, 64, 128, 256
channels, two 3x3 convolutions + ReLU per level, 2x2 average pooling) ->
decoder (nearest upsampling, 3x3 convolutions 256->128 at 32^2, 128->64 at
64^2, 64->2 linear) -> (amplitude, phase) of the central 64^2 window of the
patch.  The phase target has its circular mean removed: a pattern is blind to
a constant phase of its patch, and the stitch synchronises window phases.
Training: Adam on patterns the forward model generates from synthetic
objects, then optional fine-tuning through the differentiable operator
(Poisson deviance of the stitched object).
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import math
import time

import numpy as np
import torch

from . import nn, ptyg, synth

N_IN = 128          # pattern size
Q = 64              # predicted window
OFF = (N_IN - Q) // 2
INPUT_SCALE = 0.1

# (kind, cin, cout, relu)
LAYERS = [
    ("conv", 1, 32, True), ("conv", 32, 32, True), ("pool",),
    ("conv", 32, 64, True), ("conv", 64, 64, True), ("pool",),
    ("conv", 64, 128, True), ("conv", 128, 128, True), ("pool",),
    ("conv", 128, 256, True), ("conv", 256, 256, True),
    ("up",), ("conv", 256, 128, True),
    ("up",), ("conv", 128, 64, True),
    ("conv", 64, 2, False),
]


class Net:
    """Parameters, Adam state and the forward / backward passes."""

    def __init__(self, device, seed: int = 2106):
        rng = np.random.default_rng(seed)
        self.device = device
        self.params = []
        for spec in LAYERS:
            if spec[0] != "conv":
                self.params.append(None)
                continue
            _, cin, cout, relu = spec
            std = math.sqrt((2.0 if relu else 0.5) / (9 * cin))
            w = torch.from_numpy(rng.normal(0.0, std, (cout, 9, cin)).astype(np.float32)).to(device)
            b = torch.zeros(cout, dtype=torch.float32, device=device)
            if not relu:
                b[0] = 0.95                      # amplitude prior of the objects
            nw, nwt = nn.weight_sizes(cin, cout)
            p = {"w32": w, "b": b, "w": torch.empty(nw, dtype=torch.bfloat16, device=device),
                 "wt": torch.empty(nwt, dtype=torch.bfloat16, device=device),
                 "gw": torch.zeros_like(w), "gb": torch.zeros_like(b),
                 "mw": torch.zeros_like(w), "vw": torch.zeros_like(w),
                 "mb": torch.zeros_like(b), "vb": torch.zeros_like(b)}
            nn.pack_weights(p["w32"], cin, cout, p["w"], p["wt"])
            self.params.append(p)
        self.step_count = 0
        self._scratch = None

    def state_dict(self):
        return {f"{i}.{k}": v.detach().cpu() for i, p in enumerate(self.params) if p
                for k, v in p.items() if k in ("w32", "b")}

    def load_state_dict(self, sd):
        for i, p in enumerate(self.params):
            if p:
                p["w32"].copy_(sd[f"{i}.w32"].to(self.device))
                p["b"].copy_(sd[f"{i}.b"].to(self.device))
                _, cin, cout, _ = LAYERS[i]
                nn.pack_weights(p["w32"], cin, cout, p["w"], p["wt"])

    # ------------------------------------------------------------ forward
    def forward(self, d: torch.Tensor, keep: bool = True):
        """d: float32 [B, 128, 128] intensities -> float32 [B, 64, 64, 8]."""
        B = d.shape[0]
        x = torch.empty((B, N_IN, N_IN, 8), dtype=torch.bfloat16, device=self.device)
        nn.net_input(d.contiguous(), x, INPUT_SCALE)
        H = N_IN
        acts = [(x, H, 1)]
        for i, spec in enumerate(LAYERS):
            cur, H, c = acts[-1]
            if spec[0] == "conv":
                _, cin, cout, relu = spec
                last = i == len(LAYERS) - 1
                y = torch.empty((B, H, H, nn.cpad(cout)), dtype=torch.float32 if last else torch.bfloat16,
                                device=self.device)
                p = self.params[i]
                nn.conv_fwd(cur, p["w"], p["b"], y, B, H, H, cin, cout, relu, out_f32=last)
                acts.append((y, H, cout))
            elif spec[0] == "pool":
                y = torch.empty((B, H // 2, H // 2, nn.cpad(c)), dtype=torch.bfloat16, device=self.device)
                nn.pool2(cur, y, B, H, H, c)
                acts.append((y, H // 2, c))
            else:
                y = torch.empty((B, 2 * H, 2 * H, nn.cpad(c)), dtype=torch.bfloat16, device=self.device)
                nn.up2(cur, y, B, H, H, c)
                acts.append((y, 2 * H, c))
            if not keep and len(acts) > 2:
                acts[-2] = None
        self._acts = acts if keep else None
        return acts[-1][0]

    # ----------------------------------------------------------- backward
    def backward(self, dout: torch.Tensor):
        """dout: bf16 [B, 64, 64, 8], gradient of the loss w.r.t. the output."""
        acts = self._acts
        B = dout.shape[0]
        dy = dout
        for i in range(len(LAYERS) - 1, -1, -1):
            spec = LAYERS[i]
            x_in, H, c_in = acts[i]
            y_out, Ho, c_out = acts[i + 1]
            if spec[0] == "conv":
                _, cin, cout, relu = spec
                dz = dy
                if relu:
                    dz = torch.empty_like(dy)
                    nn.relu_bwd(dy, y_out, dz)
                p = self.params[i]
                need = nn.wgrad_scratch(B, H, H, cin, cout)
                if self._scratch is None or self._scratch.numel() < need:
                    self._scratch = torch.empty(need, dtype=torch.uint8, device=self.device)
                nn.conv_bwd_weight(x_in, dz, p["gw"], p["gb"], B, H, H, cin, cout, self._scratch)
                if i > 0:
                    dx = torch.empty((B, H, H, nn.cpad(cin)), dtype=torch.bfloat16, device=self.device)
                    nn.conv_bwd_data(dz, p["wt"], dx, B, H, H, cin, cout)
                    dy = dx
            elif spec[0] == "pool":
                dx = torch.empty((B, H, H, nn.cpad(c_in)), dtype=torch.bfloat16, device=self.device)
                nn.pool2(dy, dx, B, H, H, c_in, backward=True)
                dy = dx
            else:
                dx = torch.empty((B, H, H, nn.cpad(c_in)), dtype=torch.bfloat16, device=self.device)
                nn.up2(dy, dx, B, H, H, c_in, backward=True)
                dy = dx

    def reset_optimizer(self):
        """Zero Adam's moment estimates and step count (a new objective)."""
        self.step_count = 0
        for p in self.params:
            if p:
                for k in ("mw", "vw", "mb", "vb"):
                    p[k].zero_()

    def adam_step(self, lr: float):
        self.step_count += 1
        for i, p in enumerate(self.params):
            if not p:
                continue
            nn.adam(p["w32"], p["gw"], p["mw"], p["vw"], lr, self.step_count)
            nn.adam(p["b"], p["gb"], p["mb"], p["vb"], lr, self.step_count)
            _, cin, cout, _ = LAYERS[i]
            nn.pack_weights(p["w32"], cin, cout, p["w"], p["wt"])


# ---------------------------------------------------------------- data
def _object(seed: int, size: int):
    return synth.make_object(size, size, seed).astype(np.complex64)


def raster(size: int, grid: int, step: int, jitter: int, rng) -> np.ndarray:
    span = (grid - 1) * step + N_IN
    o_r = int(rng.integers(jitter, size - span - jitter + 1))
    o_c = int(rng.integers(jitter, size - span - jitter + 1))
    ii, jj = np.meshgrid(np.arange(grid), np.arange(grid), indexing="ij")
    r = o_r + ii * step + rng.integers(-jitter, jitter + 1, ii.shape)
    c = o_c + jj * step + rng.integers(-jitter, jitter + 1, jj.shape)
    return np.stack([r.ravel(), c.ravel()], 1).astype(np.int32)


def window_targets(obj: torch.Tensor, pos: torch.Tensor) -> torch.Tensor:
    """(amplitude, phase minus its circular mean) of the central Q^2 window of
    every patch: float32 [k, Q, Q, 2]."""
    k = pos.shape[0]
    ar = torch.arange(Q, device=obj.device)
    rows = (pos[:, 0:1].long() + OFF + ar[None, :])[:, :, None]
    cols = (pos[:, 1:2].long() + OFF + ar[None, :])[:, None, :]
    win = obj[rows, cols]                                    # [k, Q, Q] complex
    mean_phase = torch.angle(win.sum(dim=(1, 2)))
    win = win * torch.exp(-1j * mean_phase)[:, None, None]
    return torch.stack([win.abs(), torch.angle(win)], dim=-1).float().contiguous()


@dataclasses.dataclass
class TrainingSet:
    data: torch.Tensor      # float32 [n, 128, 128] Poisson counts
    target: torch.Tensor    # float32 [n, 64, 64, 2]


def make_training_set(probe: torch.Tensor, n_objects: int = 500, per_side: int = 20, size: int = 1024,
                      step: int = 24, jitter: int = 2, seed: int = synth.SEED_BASE + 4000,
                      workers: int = 8) -> TrainingSet:
    """Patterns generated by the forward model (ptyg_forward) from synthetic
    objects of `size`^2 on jittered rasters with random origins, with Poisson
    noise; the c2 probe and photon count."""
    dev = probe.device
    ds, ts = [], []
    seeds = [seed + i for i in range(n_objects)]
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        for o in ex.map(_object, seeds, [size] * n_objects):
            obj = torch.from_numpy(o).to(dev)
            pos = torch.from_numpy(raster(size, per_side, step, jitter, rng)).to(dev)
            far = ptyg.forward(obj, probe, pos)
            ds.append(torch.poisson((far.real ** 2 + far.imag ** 2).float(), generator=gen))
            ts.append(window_targets(obj, pos))
    return TrainingSet(torch.cat(ds), torch.cat(ts))


# ------------------------------------------------------------- training
def train(net: Net, ts: TrainingSet, epochs: float = 1.0, batch: int = 64, lr: float = 5e-4,
          seed: int = 7, warmup: int = 100, log=None) -> list:
    """Adam on the window MSE (learning rate: linear warm-up over `warmup`
    steps, then constant, x0.2 for the last quarter); returns the loss
    history (mean of every 10th step, per 50 steps)."""
    n = ts.data.shape[0]
    gen = torch.Generator(device=ts.data.device)
    gen.manual_seed(seed)
    steps = int(epochs * n / batch)
    nparts = 64
    parts = torch.empty(nparts, dtype=torch.float64, device=ts.data.device)
    hist = []
    perm = torch.randperm(n, generator=gen, device=ts.data.device)
    pi = 0
    acc = 0.0
    for s in range(steps):
        if pi + batch > n:
            perm = torch.randperm(n, generator=gen, device=ts.data.device)
            pi = 0
        idx = perm[pi:pi + batch]
        pi += batch
        d = ts.data.index_select(0, idx)
        t = ts.target.index_select(0, idx)
        out = net.forward(d)
        dout = torch.empty(out.shape, dtype=torch.bfloat16, device=out.device)
        nn.mse(out, t, dout, parts)
        net.backward(dout)
        net.adam_step(lr * min(1.0, (s + 1) / warmup) * (1.0 if s < 0.75 * steps else 0.2))
        acc += float(parts.sum()) / (batch * Q * Q * 2) if (s % 10 == 0) else 0.0
        if (s + 1) % 50 == 0:
            hist.append(acc / 5)
            if log:
                log(f"step {s + 1}/{steps} loss {acc / 5:.5f}")
            acc = 0.0
    return hist


def predict(net: Net, data: torch.Tensor, batch: int = 256) -> torch.Tensor:
    """Network output for every pattern: float32 [k, 64, 64, 8]."""
    outs = []
    for lo in range(0, data.shape[0], batch):
        outs.append(net.forward(data[lo:lo + batch], keep=False).clone())
    return torch.cat(outs)


class Stitcher:
    """Phase synchronisation and overlap averaging of the predicted windows
    at the scan positions of one object."""

    def __init__(self, pos: torch.Tensor, obj_shape, maxnb: int = 64, iters: int = 50):
        self.H, self.W = int(obj_shape[0]), int(obj_shape[1])
        K = pos.shape[0]
        dev = pos.device
        self.wpos = torch.empty_like(pos)
        nn.shift_positions(pos, OFF, self.wpos)
        self.offsets, self.lst = nn.tile_lists(self.wpos, self.H, self.W, Q)
        self.maxnb, self.iters = maxnb, iters
        self.scratch = {"cnt": torch.empty(K, dtype=torch.int32, device=dev),
                        "nb": torch.empty(K * maxnb, dtype=torch.int32, device=dev),
                        "c": torch.empty((K * maxnb, 2), dtype=torch.float64, device=dev),
                        "ztmp": torch.empty((K, 2), dtype=torch.float64, device=dev)}
        self.count = torch.empty((self.H, self.W), dtype=torch.int32, device=dev)
        nn.cover_count(self.wpos, self.H, self.W, Q, self.offsets, self.lst, self.count)

    def __call__(self, out: torch.Tensor):
        """(psi_0 complex64 [H, W], z) from the network output."""
        P = torch.empty(out.shape[:3], dtype=torch.complex64, device=out.device)
        nn.patches(out, P)
        z = nn.phase_sync(P, self.wpos, Q, self.maxnb, self.iters, self.scratch)
        psi0 = torch.empty((self.H, self.W), dtype=torch.complex64, device=out.device)
        nn.stitch(P, z, self.wpos, self.offsets, self.lst, self.H, self.W, Q, psi0)
        return psi0, z


def finetune(net: Net, objects, probe, steps: int = 20, lr: float = 2e-4, batch_objects: int = 1, log=None):
    """Fine-tune through the differentiable operator: the loss is the Poisson
    deviance Phi(stitch(net(d))) of each training object; its gradient
    (ptyg_grad, Eq. gradient) is pulled back through the stitch
    (ptyg_ws_stitch_adjoint, window phases held fixed) into the network.
    Adam restarts from zero moments: the second-moment estimates of the
    supervised loss would mis-scale the first steps on the new objective
    (a fine-tuning run that kept them raised the deviance, 8.3e5 -> 9.0e5)."""
    net.reset_optimizer()
    hist = []
    for s in range(steps):
        obj_i = objects[s % len(objects)]
        pos, data = obj_i["pos"], obj_i["data"]
        st = obj_i.setdefault("stitcher", Stitcher(pos, obj_i["shape"]))
        out = net.forward(data)
        psi0, z = st(out)
        objective, g, _ = ptyg.grad(psi0, probe, pos, data)
        dout = torch.empty(out.shape, dtype=torch.bfloat16, device=out.device)
        scale = 1.0 / float(data.numel())   # deviance per pixel
        nn.stitch_adjoint(g, out, z, st.wpos, st.count, st.W, Q, scale, dout)
        net.backward(dout)
        net.adam_step(lr)
        hist.append(float(objective[0]))
        if log:
            log(f"finetune step {s + 1}/{steps} Phi {hist[-1]:.6e}")
    return hist


def finetune_objects(probe, n: int = 8, size: int = 1024):
    """Fine-tuning set: n further synthetic size^2 objects (seeds apart from
    the training set's), seeded jittered rasters and Poisson counts from the
    forward model with the given probe."""
    dev = probe.device
    objs = []
    rng = np.random.default_rng(99)
    for i in range(n):
        o = torch.from_numpy(_object(synth.SEED_BASE + 9000 + i, size)).to(dev)
        p = torch.from_numpy(raster(size, 20, 24, 2, rng)).to(dev)
        far = ptyg.forward(o, probe, p)
        gen = torch.Generator(device=dev)
        gen.manual_seed(9000 + i)
        objs.append({"pos": p, "data": torch.poisson((far.real ** 2 + far.imag ** 2).float(), generator=gen)
                     .contiguous(), "shape": (size, size)})
    return objs


def thin_positions(pos, min_sep: int) -> np.ndarray:
    """Indices of a subset of the scan positions, greedy in scan order, with
    every kept pair at least `min_sep` apart in row or column.  With
    `min_sep` below the predicted window (64) the kept windows still overlap,
    so they cover the scanned area and can be phase-synchronised."""
    p = pos.cpu().numpy() if torch.is_tensor(pos) else np.asarray(pos)
    kept = np.zeros((0, 2), p.dtype)
    idx = []
    for k in range(len(p)):
        if len(kept) == 0 or np.all(np.maximum(np.abs(kept[:, 0] - p[k, 0]), np.abs(kept[:, 1] - p[k, 1])) >= min_sep):
            idx.append(k)
            kept = np.vstack([kept, p[k:k + 1]])
    return np.asarray(idx, np.int64)


def time_to_objective(net: Net, probe, pos, data, obj_shape, obj_true=None, plain_iters: int = 100,
                      max_iters: int = 200, sync_iters: int = 100, line_search: str = "batched",
                      infer_sep: int = 0):
    """Plain CG (psi_0 = 1, `plain_iters` iterations) against the warm start
    (inference + stitch + CG until its objective reaches plain CG's final
    one).  Wall times are synchronised host timings.  infer_sep > 0: the
    network sees only the patterns of thin_positions(pos, infer_sep) (the
    selection, like the stitcher's lists, is set-up and not timed)."""
    H, W = int(obj_shape[0]), int(obj_shape[1])
    K = pos.shape[0]
    sel = None
    if infer_sep > 0:
        sel = torch.from_numpy(thin_positions(pos, infer_sep)).to(pos.device)
    ws = ptyg.workspace(ptyg.dims_of((H, W), probe.shape[0], K), probe.device, line_search=line_search)
    ones = torch.ones((H, W), dtype=torch.complex64, device=probe.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = ptyg.cg_solve(ones, probe, pos, data, plain_iters, ws=ws, line_search=line_search)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    phi_plain = plain.trace[-1]["phi"] if plain.trace else float("nan")
    # the objective of plain CG's final iterate (after its last update)
    phi_plain_final = float(ptyg.minfunc(plain.obj, probe, pos, data, ws=ws)[0])
    pos_in = pos if sel is None else pos[sel].contiguous()
    data_in = data if sel is None else data[sel].contiguous()
    st = Stitcher(pos_in, (H, W), iters=sync_iters)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out = predict(net, data_in)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t1
    t2 = time.perf_counter()
    psi0, _ = st(out)
    torch.cuda.synchronize()
    t_stitch = time.perf_counter() - t2
    phi0_warm = float(ptyg.minfunc(psi0, probe, pos, data, ws=ws)[0])
    t3 = time.perf_counter()
    warm = ptyg.cg_solve(psi0, probe, pos, data, max_iters, target_phi=phi_plain_final, ws=ws,
                         line_search=line_search)
    torch.cuda.synchronize()
    t_cg = time.perf_counter() - t3
    phi_warm_final = float(ptyg.minfunc(warm.obj, probe, pos, data, ws=ws)[0])
    reached = warm.iters_done < max_iters or phi_warm_final <= phi_plain_final
    t_plain_per_iter = t_plain / max(plain.iters_done, 1)
    marks = [0, 5, 10, 25, 50, 75, 99]
    res = {"phi_plain_final": phi_plain_final, "phi_plain_last_trace": phi_plain, "t_plain_s": t_plain,
           "plain_iters": plain.iters_done, "phi0_ones": plain.trace[0]["phi"] if plain.trace else None,
           "phi0_warm": phi0_warm, "t_infer_s": t_infer, "t_stitch_s": t_stitch, "t_cg_warm_s": t_cg,
           "warm_iters": warm.iters_done, "warm_reached_target": bool(reached),
           "infer_patterns": int(K if sel is None else len(sel)),
           "t_warm_total_s": t_infer + t_stitch + t_cg, "phi_warm_final": phi_warm_final,
           "warm_faster": bool(reached) and t_infer + t_stitch + t_cg < t_plain,
           "break_even_iters": (t_plain - t_infer - t_stitch) / t_plain_per_iter,
           "phi_trace_plain": {m: plain.trace[m]["phi"] for m in marks if m < len(plain.trace)},
           "phi_trace_warm": {m: warm.trace[m]["phi"] for m in marks if m < len(warm.trace)}}
    if obj_true is not None:
        res["err_plain"] = aligned_error(plain.obj, obj_true, probe, pos)
        res["err_warm"] = aligned_error(warm.obj, obj_true, probe, pos)
        res["err_psi0_warm"] = aligned_error(psi0, obj_true, probe, pos)
    return res


def aligned_error(rec: torch.Tensor, truth: torch.Tensor, probe, pos) -> float:
    """Relative error over the illuminated region (sum_k |p|^2 placed at the
    scan positions >= 1e-3 of its maximum, obtained as G^H G 1 with the
    probe |p|) after removing the unobservable global phase."""
    pa = probe.abs().to(torch.complex64)
    illum, _ = ptyg.adjoint(ptyg.forward(torch.ones_like(truth), pa, pos), pa, pos, tuple(truth.shape))
    mask = illum.real >= 1e-3 * illum.real.max()
    s = torch.vdot(rec[mask], truth[mask])
    al = rec * torch.exp(1j * torch.angle(s))
    return float(torch.linalg.vector_norm((al - truth)[mask]) / torch.linalg.vector_norm(truth[mask]))


def heldout_projection(device):
    """The held-out projection: the 2048^2 / 128^2 / 4096-position workload
    (object, disk probe, jittered raster, Poisson counts at 1e5 photons),
    with measurements drawn by the forward model on the ground truth."""
    cfg = synth.CONFIGS["c2"]
    inp = synth.make_inputs(cfg)
    obj_true = torch.from_numpy(inp.obj_true.astype(np.complex64)).to(device)
    probe = torch.from_numpy(inp.probe.astype(np.complex64)).to(device)
    pos = torch.from_numpy(inp.pos).to(device)
    far = ptyg.forward(obj_true, probe, pos)
    gen = torch.Generator(device=device)
    gen.manual_seed(cfg.seed("poisson"))
    data = torch.poisson((far.real ** 2 + far.imag ** 2).float(), generator=gen).contiguous()
    del far
    return cfg, obj_true, probe, pos, data


def main(argv=None):
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="train the warm-start network on forward-model data and "
                                             "measure time-to-objective on the held-out projection")
    ap.add_argument("--objects", type=int, default=500)
    ap.add_argument("--per-side", type=int, default=20, help="scan raster per training object (per side)")
    ap.add_argument("--epochs", type=float, default=1.0)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--finetune", type=int, default=400, help="fine-tuning steps through the operator")
    ap.add_argument("--finetune-lr", type=float, default=3e-4)
    ap.add_argument("--sync-iters", type=int, default=100)
    ap.add_argument("--infer-sep", type=int, default=40,
                    help="infer only a subset of patterns at least this many pixels apart (0: all)")
    ap.add_argument("--line-search", default="batched", choices=["batched", "sequential"])
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    cfg, obj_true, probe, pos, data = heldout_projection(dev)
    t0 = time.perf_counter()
    ts = make_training_set(probe, n_objects=args.objects, per_side=args.per_side)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"training set: {ts.data.shape[0]} patterns in {t_data:.1f} s")
    net = Net(dev)
    t1 = time.perf_counter()
    hist = train(net, ts, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    del ts
    ft = []
    t_ft = 0.0
    if args.finetune:
        t2 = time.perf_counter()
        objs = finetune_objects(probe)
        ft = finetune(net, objs, probe, steps=args.finetune, lr=args.finetune_lr)
        torch.cuda.synchronize()
        t_ft = time.perf_counter() - t2
        log(f"fine-tuned {args.finetune} steps in {t_ft:.1f} s: Phi {ft[0]:.4e} -> {ft[-1]:.4e}")
    res = time_to_objective(net, probe, pos, data, tuple(obj_true.shape), obj_true, sync_iters=args.sync_iters,
                            line_search=args.line_search, infer_sep=args.infer_sep)
    res.update({"train_patterns": args.objects * args.per_side ** 2, "train_epochs": args.epochs,
                "t_data_s": round(t_data, 2), "t_train_s": round(t_train, 2), "loss_history": hist[-5:],
                "finetune_steps": args.finetune, "t_finetune_s": round(t_ft, 2),
                "finetune_phi_first_last": [ft[0], ft[-1]] if ft else None,
                "workload": "held-out 2048^2 object, 128^2 disk probe, 4096 positions, Poisson 1e5"})
    print(json.dumps(res))


if __name__ == "__main__":
    main()
