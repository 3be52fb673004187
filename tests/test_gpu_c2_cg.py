"""ML-CG at the full single-projection workload for the stated 100
iterations (2048^2 object, 128^2 probe, 4096 positions, Poisson at 1e5
photons; Algorithm 1, Eqs. update, DaiYuan, linesearch), both line-search
modes, against the oracle's traces in tests/golden/ (written by
tests/golden/make_c2_trace.py from the oracle alone: FP64, and with every
transform rounded to FP32).

* Decisions: identical step and accepted trial in every iteration up to a
  first disagreement, which must be legitimate (_cases.agreed_iterations:
  a tie of the sufficient-decrease test, or a Dai-Yuan coefficient the
  FP32-transform oracle already moves by 1% or more).
* Iterates: on ten fixed 16 x 16 windows after iterations 1, 10 and 100,
  relative L2 within max(1e-3, c x) the FP32-transform oracle's distance
  from the FP64 one on the same windows, c the gradient-bound factor at the
  start (_cases.trajectory_factor).  Before a first disagreement this is the
  first-order bound that trajectory_factor documents (per-step perturbations
  at most c times the FP32 floor's).  After a legitimate one the oracle's FP32-transform run is
  itself a trajectory that parted from the FP64 one at an indeterminate
  decision, and its distance at the same iteration is the band an FP32
  implementation lands in; the same factor c applies.  On this workload the
  FP32-transform run parts at iteration 3 (its Dai-Yuan coefficient moves by
  27%), so every FP32 solver is held to that band from there on.
* The first step's 2-norm (Results' convergence metric) within the gradient
  bound; a monotone objective; the final objective no higher than the
  oracle's by more than 1e-3 relative.  The window errors at every stored
  iteration, the first disagreement and the error against the ground truth
  are printed."""
import json
import os

import numpy as np
import pytest

from oracle import ptycho as O

from _cases import agreed_iterations, grad_bound, rel, trajectory_factor, workload
from _gpu import dev, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def P():
    return lib()


@pytest.fixture(scope="module")
def gold():
    g64 = json.load(open(os.path.join(GOLD, "c2_trace_fp64.json")))
    g32 = json.load(open(os.path.join(GOLD, "c2_trace_fp32t.json")))
    return g64, g32


@pytest.fixture(scope="module")
def factor(P):
    cfg, inp, probe, obj, data = workload("c2")
    psi = np.ones(obj.shape, np.complex64)
    far = P.forward(dev(psi), dev(probe), dev(inp.pos)).cpu().numpy()
    _, bo, _, fo, _ = grad_bound(far, psi, probe, inp.pos, data)
    print(f"c2 start: gradient bound {bo:.2e}, fp32 floor {fo:.2e}")
    return bo, trajectory_factor(bo, fo)


def windows(x, g):
    w = g["window"]
    return np.stack([x[r:r + w, c:c + w] for r, c in g["window_corners"]])


def gold_windows(g, m):
    return np.array([np.array(re) + 1j * np.array(im) for re, im in g["snapshots"][str(m)]["windows"]])


@pytest.mark.parametrize("ls", ["sequential", "batched"])
def test_c2_cg_100_iterations(P, gold, factor, ls):
    g64, g32 = gold
    bo, c = factor
    cfg, inp, probe, obj, data = workload("c2")
    iters = g64["iters"]
    args = (dev(np.ones(obj.shape, np.complex64)), dev(probe), dev(inp.pos), dev(data))
    res = P.cg_solve(*args, iters, line_search=ls)
    tr = res.trace
    assert res.iters_done == iters
    same, why = agreed_iterations(tr, g64["trace"], g32["trace"])
    print(f"c2 {ls}: decisions agree for {same} of {iters} iterations" + (f"; {why}" if why else ""))
    # objective: monotone, first value to the objective bar, final level
    phis = [r["phi"] for r in tr]
    assert all(b <= a for a, b in zip(phis, phis[1:]))
    assert abs(phis[0] - g64["trace"][0]["phi"]) <= 1e-5 * g64["trace"][0]["phi"]
    print(f"   final phi gpu {phis[-1]:.8e} oracle {g64['trace'][-1]['phi']:.8e} "
          f"fp32-transform oracle {g32['trace'][-1]['phi']:.8e}")
    assert phis[-1] <= g64["trace"][-1]["phi"] * (1 + 1e-3)
    # the first update's 2-norm: gamma_0 ||grad(psi_0)||
    sn, sn_o = tr[0]["step_norm"], g64["trace"][0]["step_norm"]
    assert abs(sn - sn_o) <= max(bo, 1e-5) * sn_o
    # iterates on the sample windows
    truth = obj.astype(np.complex128)
    illum = O.illumination(probe.astype(np.complex128), inp.pos, obj.shape)
    mask = illum >= 1e-3 * illum.max()
    for m in (1, 10, 100):
        r = res if m == iters else P.cg_solve(*args, m, line_search=ls)
        got = windows(r.obj.cpu().numpy(), g64)
        e = rel(got, gold_windows(g64, m))
        floor = rel(gold_windows(g32, m), gold_windows(g64, m))
        al = O.align_phase(r.obj.cpu().numpy().astype(np.complex128), truth, mask)
        et = rel(al[mask], truth[mask])
        print(f"   after {m}: windows rel {e:.2e} (fp32 floor {floor:.2e}, bound {max(1e-3, c * floor):.2e}); "
              f"error vs truth gpu {et:.4e} oracle {g64['snapshots'][str(m)]['err_vs_truth']:.4e}")
        assert e <= max(1e-3, c * floor)
