"""Least-squares estimator (estimator="ls") on the GPU against the oracle:
the same bars as the Poisson path (objectives 1e-5, gradients within the
bound their forward error implies through the residual's conditioning, CG
and GD iterates within the iterate bound of _cases.trajectory_factor,
identical line-search decisions on well-conditioned workloads)."""
import numpy as np
import pytest

from oracle import ptycho as O

from _cases import cg_with_floor, gd_with_floor, grad_bound, rel, workload
from _gpu import start_factors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
LS = "ls"


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_07575_amd import ptyg
    ptyg.load()
    return ptyg


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def start(obj):
    # between psi0 = 1 and the truth, so that residuals are neither zero nor huge
    return (0.7 * np.ones(obj.shape) + 0.3 * obj).astype(np.complex64)


@pytest.mark.parametrize("case", ["c1", "m32", "m16r", "m128", "m256"])
def test_ls_grad_and_objective(P, case):
    cfg, inp, probe, obj, data = workload(case)
    psi = start(obj)
    print(f"ls grad {case}", flush=True)
    objective, g, gp = P.grad(dev(psi), dev(probe), dev(inp.pos), dev(data), want_probe=True, estimator=LS)
    far = P.forward(dev(psi), dev(probe), dev(inp.pos)).cpu().numpy()
    ref, bo, bp, fo, fp = grad_bound(far, psi, probe, inp.pos, data, want_probe=True, estimator=LS)
    eo, ep = rel(g.cpu().numpy(), ref["grad_obj"]), rel(gp.cpu().numpy(), ref["grad_probe"])
    print(f"   grad obj rel {eo:.2e} (bound {bo:.2e}, floor {fo:.2e}) probe {ep:.2e} (bound {bp:.2e}, floor {fp:.2e})")
    assert eo <= bo and ep <= bp
    ob = objective.cpu().numpy()
    assert abs(ob[0] - ref["phi"]) <= 1e-5 * ref["phi"] and abs(ob[1] - ref["f"]) <= 1e-5 * ref["f"]
    mf = P.minfunc(dev(psi), dev(probe), dev(inp.pos), dev(data), estimator=LS).cpu().numpy()
    assert abs(mf[0] - ref["phi"]) <= 1e-5 * ref["phi"]


@pytest.mark.parametrize("ls", ["sequential", "batched"])
@pytest.mark.parametrize("case,iters", [("m32", 8), ("m16r", 8)])
def test_ls_cg_well_conditioned_exact_decisions(P, case, iters, ls):
    cfg, inp, probe, obj, data = workload(case)
    obj0 = np.ones(obj.shape, np.complex64)
    res = P.cg_solve(dev(obj0), dev(probe), dev(inp.pos), dev(data), iters, line_search=ls, estimator=LS)
    (ro, rp, rtr), _ = cg_with_floor(obj0, probe, inp.pos, data, iters, estimator=LS)
    err = rel(res.obj.cpu().numpy(), ro)
    print(f"ls cg {case} {ls}: object rel {err:.2e}", [r["gamma"] for r in res.trace])
    assert [r["gamma"] for r in res.trace] == [r["gamma"] for r in rtr]
    for a, b in zip(res.trace, rtr):
        assert abs(a["phi"] - b["phi"]) <= 1e-5 * abs(b["phi"])
    assert err <= 1e-3


@pytest.mark.parametrize("ls", ["sequential", "batched"])
@pytest.mark.parametrize("case,iters", [("c1", 16), ("m128", 6), ("m256", 3)])
def test_ls_cg_within_fp32_floor(P, case, iters, ls):
    cfg, inp, probe, obj, data = workload(case)
    obj0 = np.ones(obj.shape, np.complex64)
    res = P.cg_solve(dev(obj0), dev(probe), dev(inp.pos), dev(data), iters, line_search=ls, estimator=LS)
    (ro, rp, rtr), (po, pp, ptr) = cg_with_floor(obj0, probe, inp.pos, data, iters, estimator=LS)
    illum = O.illumination(probe.astype(np.complex128), inp.pos, obj.shape)
    mask = illum >= 1e-3 * illum.max()
    err, floor = rel(res.obj.cpu().numpy()[mask], ro[mask]), rel(po[mask], ro[mask])
    print(f"ls cg {case}/{iters} {ls}: object rel {err:.2e} (floor {floor:.2e})")
    c, _ = start_factors(P, obj0, probe, inp.pos, data, estimator=LS)
    assert err <= max(1e-3, c * floor)
    assert res.trace[0]["gamma"] == rtr[0]["gamma"]
    phis = [r["phi"] for r in res.trace]
    assert all(b <= a for a, b in zip(phis, phis[1:]))


def test_ls_gd(P):
    cfg, inp, probe, obj, data = workload("m32")
    obj0 = np.ones(obj.shape, np.complex64)
    gamma = 0.1 / O.illumination(probe.astype(np.complex128), inp.pos, obj.shape).max()
    o, _, phis = P.gd_solve(dev(obj0), dev(probe), dev(inp.pos), dev(data), 6, gamma, estimator=LS)
    (ro, rp, rtr), (po, pp, ptr) = gd_with_floor(obj0, probe, inp.pos, data, 6, gamma, estimator=LS)
    err, floor = rel(o.cpu().numpy(), ro), rel(po, ro)
    print(f"ls gd: object rel {err:.2e} (floor {floor:.2e})")
    c, _ = start_factors(P, obj0, probe, inp.pos, data, estimator=LS)
    assert err <= max(1e-4, c * floor)


def test_bad_estimator_is_rejected(P):
    cfg, inp, probe, obj, data = workload("c1")
    o = dev(np.ones(obj.shape, np.complex64))
    d = P.dims_of(obj.shape, probe.shape[0], inp.pos.shape[0])
    ws = P.workspace(d, torch.device("cuda"))
    g = torch.empty_like(o)
    import ctypes
    st = P.load().ptyg_grad(ctypes.byref(d), P._ptr(o), P._ptr(dev(probe)), P._ptr(dev(inp.pos)), P._ptr(dev(data)),
                            1e-32, 7, P._ptr(g), None, None, P._ptr(ws), ws.numel(), P._stream())
    assert st == -1
