"""Writes the c2 CG golden traces from the FP64 oracle (and nothing else).

Workload: the seeded single-projection case (2048^2 object, 128^2 probe,
64 x 64 = 4096 jittered positions, Poisson intensities at 1e5 photons;
intensities from the oracle's forward model, counts from the seeded
generator), object-only ML-CG from psi_0 = 1 for 100 iterations with
Algorithm 1's sequential line search (gamma0 = 1, tau = 0.5, t = 0, 40
trials at most).

Two runs:
  fp64   the oracle as it stands (complex128 throughout);
  fp32t  the same with every forward and inverse transform rounded once to
         single precision (tests/_cases.fp32_transforms): the trajectory of
         an exactly rounded FP32-transform implementation, which bounds how
         far any FP32-transform solver can follow the FP64 one.

Each output file holds the per-iteration trace (Phi, F, gamma, trial index,
beta, step norm, restart, every line-search trial's objective) and the iterate on ten fixed 16 x 16 sample windows
after iterations 1, 10 and 100, plus the illuminated-mask norm of the object
after iterations 1, 2, 5, 10, 20, 50 and 100 and the phase-aligned masked error against
the ground truth.

    python tests/golden/make_c2_trace.py fp64     # ~80 min on 8 cores
    python tests/golden/make_c2_trace.py fp32t
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

import numpy as np  # noqa: E402

from oracle import ptycho as O  # noqa: E402
from _cases import fp32_transforms, workload  # noqa: E402

ITERS = 100
RECORD = (1, 2, 5, 10, 20, 50, 100)
WINDOW_ITERS = (1, 10, 100)
WIN = 16
# top-left corners of the sample windows: a 3 x 3 grid over the scanned
# area (rows and columns 204 ... 1844) plus its centre
WINDOWS = [(r, c) for r in (420, 1008, 1596) for c in (420, 1008, 1596)] + [(1130, 880)]


def windows_of(obj):
    return [obj[r:r + WIN, c:c + WIN] for r, c in WINDOWS]


def _f32(a):
    # 9 significant digits: float32 round trip, ample for 1e-3 comparisons
    return [[float(f"{v:.9g}") for v in row] for row in np.asarray(a).tolist()]


def main(kind: str) -> None:
    cfg, inp, probe, obj_true, data = workload("c2")
    p64 = probe.astype(np.complex128)
    d64 = data.astype(np.float64)
    illum = O.illumination(p64, inp.pos, obj_true.shape)
    mask = illum >= 1e-3 * illum.max()
    truth = obj_true.astype(np.complex128)
    snaps = {}
    t0 = time.time()

    def cb(m, o, _p):
        print(f"[{kind}] iteration {m} done, {time.time() - t0:.0f} s", flush=True)
        if m in RECORD:
            al = O.align_phase(o, truth, mask)
            snaps[m] = {
                "windows": ([[_f32(w.real), _f32(w.imag)] for w in windows_of(o)]
                            if m in WINDOW_ITERS else None),
                "mask_norm": float(np.linalg.norm(o[mask])),
                "err_vs_truth": float(np.linalg.norm((al - truth)[mask]) / np.linalg.norm(truth[mask])),
            }

    psi0 = np.ones(obj_true.shape, np.complex128)
    args = (psi0, p64, inp.pos, d64, ITERS)
    if kind == "fp64":
        _, _, trace = O.cg_solve(*args, callback=cb)
    elif kind == "fp32t":
        with fp32_transforms():
            _, _, trace = O.cg_solve(*args, callback=cb)
    else:
        raise SystemExit(f"unknown kind {kind!r}")
    out = {
        "what": f"oracle ML-CG on the c2 workload, {kind}, sequential line search",
        "iters": ITERS,
        "opts": {"gamma0": 1.0, "tau": 0.5, "t": 0.0, "lmax": 40, "eps": O.EPS},
        "window": WIN,
        "window_corners": WINDOWS,
        "mask_pixels": int(mask.sum()),
        "trace": [{k: (bool(v) if k == "restarted" else (int(v) if k == "halvings" else
                       ([float(x) for x in v] if k == "trial_phis" else float(v))))
                   for k, v in row.items()} for row in trace],
        "snapshots": {str(m): snaps[m] for m in RECORD if m in snaps},
        "seconds": time.time() - t0,
    }
    path = os.path.join(HERE, f"c2_trace_{kind}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, separators=(",", ":"))
    os.replace(path + ".tmp", path)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "fp64")
