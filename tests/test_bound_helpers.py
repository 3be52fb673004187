"""The gradient-bound helpers of the parity tests agree with each other
(CPU only): grad_bound_from, fed the oracle figures grad_bound itself
computes, gives grad_bound's object and probe bounds and floors."""
import numpy as np

from oracle import ptycho as O

from _cases import fp32_transforms, grad_bound, grad_bound_from, rel, workload


def test_grad_bound_from_matches_grad_bound():
    cfg, inp, probe, obj, data = workload("m32")
    psi = np.ones(obj.shape, np.complex64)
    p0 = np.abs(probe).astype(np.complex64)
    # a stand-in FP32 far field: the oracle's, rounded to complex64
    far = O.forward(psi.astype(np.complex128), p0.astype(np.complex128), inp.pos).astype(np.complex64)
    ref, bo, bp, fo, fp = grad_bound(far, psi, p0, inp.pos, data, want_probe=True)
    with fp32_transforms():
        pert = O.grad(psi.astype(np.complex128), p0.astype(np.complex128), inp.pos, data.astype(np.float64),
                      want_probe=True)
    acc = np.sum(np.abs(O.gather(psi.astype(np.complex128), inp.pos, cfg.n)) ** 2, axis=0)
    start = {"grad_obj_norm": float(np.linalg.norm(ref["grad_obj"])),
             "grad_probe_norm": float(np.linalg.norm(ref["grad_probe"])),
             "floor_obj": rel(pert["grad_obj"], ref["grad_obj"]),
             "floor_probe": rel(pert["grad_probe"], ref["grad_probe"]),
             "lip_obj": float(np.sqrt(O.illumination(p0.astype(np.complex128), inp.pos, obj.shape).max())),
             "lip_probe": float(np.sqrt(acc.max()))}
    bo2, bp2, fo2, fp2 = grad_bound_from(far, psi, p0, inp.pos, data, start)
    assert np.isclose(bo2, bo, rtol=1e-12) and np.isclose(bp2, bp, rtol=1e-12)
    assert fo2 == fo and fp2 == fp
    assert bo > 1e-5 and bp > 1e-5
