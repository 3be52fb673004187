"""Writes the c5 joint CG golden traces from the FP64 oracle (and nothing else).

Workload: the seeded large one-GPU share (8192^2 object, 256^2 apodised-disk
probe, 128 x 128 = 16384 jittered positions on a 48 px raster, Poisson
intensities at 1e6 photons; intensities from the oracle's forward model,
counts from the seeded generator), joint object+probe ML-CG from psi_0 = 1
and the probe's amplitude |p| (its phase unknown), Algorithm 1's sequential
line search (gamma0 = 1, tau = 0.5, t = 0, 40 trials at most), ITERS
iterations.

Two runs, as for the single-projection traces:
  fp64   the oracle as it stands;
  fp32t  every forward and inverse transform rounded once to single
         precision (tests/_cases.fp32_transforms).

Each file holds the per-iteration trace (Phi, F, gamma, trial index, beta,
step norm, restart, every trial's objective), the object on ten 16 x 16
windows and the probe on four 16 x 16 windows after every iteration, and
the illuminated-mask norm of the object.  The counts (integers below 2^24)
are kept in float32, exact, to halve the memory.

    python tests/golden/make_c5_trace.py fp64     # ~1 h on 8 cores
    python tests/golden/make_c5_trace.py fp32t
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

ITERS = 2
WIN = 16
# object windows: a 3 x 3 grid over the scanned area (rows and columns
# 917 ... 7275) plus one off the grid
WINDOWS = [(r, c) for r in (1500, 4000, 6500) for c in (1500, 4000, 6500)] + [(3333, 5111)]
# probe windows: the centre, inside the disk, its edge, and the apodised tail
PROBE_WINDOWS = [(120, 120), (80, 150), (60, 120), (10, 10)]


def _f32(a):
    return [[float(f"{v:.9g}") for v in row] for row in np.asarray(a).tolist()]


def _win(x, corners):
    return [[_f32(x[r:r + WIN, c:c + WIN].real), _f32(x[r:r + WIN, c:c + WIN].imag)] for r, c in corners]


def main(kind: str) -> None:
    cfg, inp, probe, obj_true, data = workload("c5")
    p64 = probe.astype(np.complex128)
    illum = O.illumination(p64, inp.pos, obj_true.shape)
    mask = illum >= 1e-3 * illum.max()
    del illum
    snaps = {}
    t0 = time.time()

    def cb(m, o, p):
        print(f"[{kind}] iteration {m} done, {time.time() - t0:.0f} s", flush=True)
        snaps[m] = {"object_windows": _win(o, WINDOWS), "probe_windows": _win(p, PROBE_WINDOWS),
                    "mask_norm": float(np.linalg.norm(o[mask])), "probe_norm": float(np.linalg.norm(p))}

    psi0 = np.ones(obj_true.shape, np.complex128)
    args = (psi0, np.abs(p64).astype(np.complex128), inp.pos, data, ITERS)
    if kind == "fp64":
        _, _, trace = O.cg_solve(*args, update_probe=True, callback=cb)
    elif kind == "fp32t":
        with fp32_transforms():
            _, _, trace = O.cg_solve(*args, update_probe=True, callback=cb)
    else:
        raise SystemExit(f"unknown kind {kind!r}")
    out = {
        "what": f"oracle joint ML-CG on the c5 workload from psi_0 = 1 and |p|, {kind}, sequential line search",
        "iters": ITERS,
        "opts": {"gamma0": 1.0, "tau": 0.5, "t": 0.0, "lmax": 40, "eps": O.EPS},
        "window": WIN,
        "window_corners": WINDOWS,
        "probe_window_corners": PROBE_WINDOWS,
        "mask_pixels": int(mask.sum()),
        "trace": [{k: (bool(v) if k == "restarted" else (int(v) if k == "halvings" else
                       ([float(x) for x in v] if k == "trial_phis" else float(v))))
                   for k, v in row.items()} for row in trace],
        "snapshots": {str(m): snaps[m] for m in sorted(snaps)},
        "seconds": time.time() - t0,
    }
    path = os.path.join(HERE, f"c5_trace_{kind}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, separators=(",", ":"))
    os.replace(path + ".tmp", path)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "fp64")
