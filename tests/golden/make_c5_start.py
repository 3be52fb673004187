"""Writes the oracle's gradient figures at the start of the large one-GPU
share's joint CG (8192^2 object, 256^2 probe, 16384 positions, Poisson at
1e6 photons; psi_0 = 1, probe |p|) from the oracle alone: the object and
probe gradient norms (Eq. gradient), the FP32 floors (the same gradients
with every transform rounded once to single precision, relative to the
FP64 ones), and the Lipschitz constants of G^H for the two blocks
(sqrt of the largest illumination, sqrt of the largest sum over patterns
of |psi|^2 under the probe).  With them a test bounds an FP32 gradient from
its residual difference alone (tests/_cases.grad_bound_from), without
recomputing two full oracle gradients.

    python tests/golden/make_c5_start.py     # ~15 min on 8 cores
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
from _cases import fp32_transforms, rel, workload  # noqa: E402


def main() -> None:
    t0 = time.time()
    cfg, inp, probe, obj_true, data = workload("c5")
    psi = np.ones(obj_true.shape, np.complex128)
    p0 = np.abs(probe.astype(np.complex128)).astype(np.complex128)
    ref = O.grad(psi, p0, inp.pos, data, want_probe=True)
    print(f"FP64 gradient done, {time.time() - t0:.0f} s", flush=True)
    with fp32_transforms():
        pert = O.grad(psi, p0, inp.pos, data, want_probe=True)
    print(f"FP32-transform gradient done, {time.time() - t0:.0f} s", flush=True)
    n = cfg.n
    acc = np.zeros((n, n))
    for lo in range(0, cfg.k, 256):
        acc += np.sum(np.abs(O.gather(psi, inp.pos[lo:lo + 256], n)) ** 2, axis=0)
    out = {
        "what": "oracle gradient figures at psi_0 = 1, probe |p|, on the c5 workload",
        "phi": ref["phi"],
        "grad_obj_norm": float(np.linalg.norm(ref["grad_obj"])),
        "grad_probe_norm": float(np.linalg.norm(ref["grad_probe"])),
        "floor_obj": rel(pert["grad_obj"], ref["grad_obj"]),
        "floor_probe": rel(pert["grad_probe"], ref["grad_probe"]),
        "lip_obj": float(np.sqrt(O.illumination(p0, inp.pos, psi.shape).max())),
        "lip_probe": float(np.sqrt(acc.max())),
        "seconds": time.time() - t0,
    }
    path = os.path.join(HERE, "c5_start.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: {out}", flush=True)


if __name__ == "__main__":
    main()
