"""GPU-side helpers of the parity tests: the library handle, host -> device
copies, and the iterate-bound factors of _cases computed at a start point."""
import numpy as np
import pytest

from _cases import grad_bound, trajectory_factor

torch = pytest.importorskip("torch")


def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_07575_amd import ptyg
    ptyg.load()
    return ptyg


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def start_factors(P, obj0, probe, pos, data, want_probe=False, estimator="ml"):
    """(object factor, probe factor or None): trajectory_factor of the
    gradient bound and the FP32 floor at the solver's start (obj0, probe)."""
    far = P.forward(dev(obj0), dev(probe), dev(pos)).cpu().numpy()
    _, bo, bp, fo, fp = grad_bound(far, obj0, probe, pos, data, want_probe=want_probe, estimator=estimator)
    co = trajectory_factor(bo, fo)
    cp = trajectory_factor(bp, fp) if want_probe else None
    print(f"   start: gradient bound {bo:.2e} (floor {fo:.2e}) -> iterate factor {co:.2f}"
          + (f"; probe bound {bp:.2e} (floor {fp:.2e}) -> {cp:.2f}" if want_probe else ""))
    return co, cp
