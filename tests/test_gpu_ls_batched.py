"""Batched line search (line_search="batched") against the oracle's CG and
the sequential GPU search.

G is linear, so a trial's far field G(psi + g eta) equals G psi + g G eta in
exact arithmetic (joint mode: (p + g dp)(psi + g eta) adds g^2 G(dp, eta)).
The batched search evaluates the trials from those stored far fields and
accepts the first that passes, so its step sequence must equal the
sequential one wherever the decisions are not within FP32 rounding of a tie:
the same bars as the sequential tests (identical steps on well-conditioned
workloads, the object bound of _cases.trajectory_factor elsewhere)."""
import numpy as np
import pytest

from oracle import ptycho as O

from _cases import cg_with_floor, rel, workload
from _gpu import start_factors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

B = "batched"


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_07575_amd import ptyg
    ptyg.load()
    return ptyg


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def mask_of(probe, pos, shape):
    illum = O.illumination(probe.astype(np.complex128), pos, shape)
    return illum >= 1e-3 * illum.max()


def run(P, case, iters, probe0=None, **kw):
    cfg, inp, probe, obj, data = workload(case)
    obj0 = np.ones(obj.shape, np.complex64)
    p0 = probe if probe0 is None else probe0
    print(f"batched LS {case} {iters} it {kw}", flush=True)
    res = P.cg_solve(dev(obj0), dev(p0), dev(inp.pos), dev(data), iters, line_search=B, **kw)
    okw = {k: v for k, v in kw.items() if k in ("gamma0", "tau", "t", "update_probe", "target_phi")}
    if "max_halvings" in kw:
        okw["lmax"] = kw["max_halvings"]
    ref, pert = cg_with_floor(obj0, p0, inp.pos, data, iters, **okw)
    return res, ref, pert, mask_of(probe, inp.pos, obj.shape)


def factors(P, case, probe0=None, joint=False):
    """Iterate-bound factors (object, probe) of the solver started at
    psi_0 = 1 and probe0 (_cases.trajectory_factor)."""
    cfg, inp, probe, obj, data = workload(case)
    p0 = probe if probe0 is None else probe0
    return start_factors(P, np.ones(obj.shape, np.complex64), p0, inp.pos, data, want_probe=joint)


def gammas(tr):
    return [r["gamma"] for r in tr]


@pytest.mark.parametrize("case,iters", [("m32", 8), ("m16r", 8)])
def test_batched_well_conditioned_exact_decisions(P, case, iters):
    res, (ro, rp, rtr), (po, pp, ptr), mask = run(P, case, iters)
    err = rel(res.obj.cpu().numpy()[mask], ro[mask])
    print(f"{case}: object rel {err:.2e}")
    assert res.iters_done == iters
    assert gammas(res.trace) == gammas(rtr)
    assert [r["halvings"] for r in res.trace] == [r["halvings"] for r in rtr]
    assert [r["restarted"] for r in res.trace] == [r["restarted"] for r in rtr]
    for a, b in zip(res.trace, rtr):
        assert abs(a["phi"] - b["phi"]) <= 1e-5 * abs(b["phi"])
    assert err <= 1e-3


@pytest.mark.parametrize("case,iters", [("c1", 32), ("m128", 10), ("m256", 4)])
def test_batched_object_within_fp32_floor(P, case, iters):
    res, (ro, rp, rtr), (po, pp, ptr), mask = run(P, case, iters)
    err = rel(res.obj.cpu().numpy()[mask], ro[mask])
    floor = rel(po[mask], ro[mask])
    print(f"{case}/{iters}: object rel {err:.2e}; fp32 floor {floor:.2e}")
    assert res.iters_done == iters
    c, _ = factors(P, case)
    assert err <= max(1e-3, c * floor)
    assert res.trace[0]["gamma"] == rtr[0]["gamma"]
    phis = [r["phi"] for r in res.trace]
    assert all(b <= a for a, b in zip(phis, phis[1:]))
    cfg, inp, probe, obj, data = workload(case)
    truth = obj.astype(np.complex128)
    e_gpu = rel(O.align_phase(res.obj.cpu().numpy().astype(np.complex128), truth, mask)[mask], truth[mask])
    e_ora = rel(O.align_phase(ro, truth, mask)[mask], truth[mask])
    print(f"   error vs truth: gpu {e_gpu:.4e} oracle {e_ora:.4e}")
    # the phase-aligned error is a minimum over phases, so it can exceed the
    # oracle's by at most the iterate difference (triangle inequality)
    slack = np.linalg.norm((res.obj.cpu().numpy() - ro)[mask]) / np.linalg.norm(truth[mask])
    assert e_gpu <= e_ora + slack * (1 + 1e-6)


@pytest.mark.parametrize("case", ["m32", "m64", "m128"])
def test_batched_equals_sequential_steps(P, case):
    """Same workload, both GPU searches: identical step sequences over the
    first iterations (before FP32 chaos can separate the trajectories).  The
    two trajectories are separate FP32 realisations (the GRAD variant that
    stores G psi rounds in its own order), so their objectives agree to the
    per-operator objective bar, 1e-5."""
    cfg, inp, probe, obj, data = workload(case)
    o0 = dev(np.ones(obj.shape, np.complex64))
    args = (o0, dev(probe), dev(inp.pos), dev(data), 4)
    rs = P.cg_solve(*args, line_search="sequential")
    rb = P.cg_solve(*args, line_search=B)
    print(case, gammas(rs.trace), gammas(rb.trace))
    assert gammas(rs.trace) == gammas(rb.trace)
    assert [r["halvings"] for r in rs.trace] == [r["halvings"] for r in rb.trace]
    for a, b in zip(rs.trace, rb.trace):
        assert abs(a["phi"] - b["phi"]) <= 1e-5 * abs(a["phi"])


def test_batched_multi_pass_search(P):
    """gamma0 = 2^24: the first acceptable trial lies past 16, so the search
    takes several passes (and the first pass is sized from no history)."""
    res, (ro, rp, rtr), _, mask = run(P, "m32", 4, gamma0=2.0 ** 24)
    print("halvings", [r["halvings"] for r in res.trace], [r["halvings"] for r in rtr])
    assert res.trace[0]["halvings"] > 16
    assert gammas(res.trace) == gammas(rtr)


def test_batched_restart_after_failed_search(P):
    res, (ro, rp, rtr), _, mask = run(P, "c1", 3, gamma0=1e9, max_halvings=1)
    assert res.trace[0]["gamma"] == 0.0 and rtr[0]["gamma"] == 0.0
    assert res.trace[0]["halvings"] == 1
    assert res.trace[1]["restarted"] and rtr[1]["restarted"]
    assert gammas(res.trace) == gammas(rtr)


def test_batched_joint_probe(P):
    cfg, inp, probe, obj, data = workload("m16r")
    p0 = (np.abs(probe) * np.exp(0.2j)).astype(np.complex64)
    res, (ro, rp, rtr), (po, pp, ptr), mask = run(P, "m16r", 6, probe0=p0, update_probe=True)
    co, cp = factors(P, "m16r", probe0=p0, joint=True)
    eo = rel(res.obj.cpu().numpy()[mask], ro[mask])
    ep = rel(res.probe.cpu().numpy(), rp)
    fo, fp = rel(po[mask], ro[mask]), rel(pp, rp)
    print(f"joint: object rel {eo:.2e} (floor {fo:.2e}) probe rel {ep:.2e} (floor {fp:.2e})")
    assert gammas(res.trace) == gammas(rtr)
    assert eo <= max(1e-3, co * fo)
    assert ep <= max(1e-3, cp * fp)


def test_batched_joint_probe_128(P):
    """n = 128 joint: full far fields, coefficients over the patches."""
    cfg, inp, probe, obj, data = workload("m128")
    rng = np.random.default_rng(4)
    p0 = (probe * (1 + 0.05 * rng.standard_normal(probe.shape))).astype(np.complex64)
    res, (ro, rp, rtr), (po, pp, ptr), mask = run(P, "m128", 4, probe0=p0, update_probe=True)
    co, cp = factors(P, "m128", probe0=p0, joint=True)
    eo = rel(res.obj.cpu().numpy()[mask], ro[mask])
    ep = rel(res.probe.cpu().numpy(), rp)
    fo, fp = rel(po[mask], ro[mask]), rel(pp, rp)
    print(f"joint 128: object rel {eo:.2e} (floor {fo:.2e}) probe rel {ep:.2e} (floor {fp:.2e})")
    assert gammas(res.trace) == gammas(rtr)
    assert eo <= max(1e-3, co * fo)
    assert ep <= max(1e-3, cp * fp)


def test_batched_joint_probe_256(P):
    cfg, inp, probe, obj, data = workload("m256")
    rng = np.random.default_rng(3)
    p0 = (probe * (1 + 0.05 * rng.standard_normal(probe.shape))).astype(np.complex64)
    res, (ro, rp, rtr), (po, pp, ptr), mask = run(P, "m256", 3, probe0=p0, update_probe=True)
    co, cp = factors(P, "m256", probe0=p0, joint=True)
    eo = rel(res.obj.cpu().numpy()[mask], ro[mask])
    ep = rel(res.probe.cpu().numpy(), rp)
    fo, fp = rel(po[mask], ro[mask]), rel(pp, rp)
    print(f"joint 256: object rel {eo:.2e} (floor {fo:.2e}) probe rel {ep:.2e} (floor {fp:.2e})")
    assert gammas(res.trace) == gammas(rtr)
    assert eo <= max(1e-3, co * fo)
    assert ep <= max(1e-3, cp * fp)


def test_batched_is_bit_reproducible(P):
    cfg, inp, probe, obj, data = workload("m128")
    o0 = dev(np.ones(obj.shape, np.complex64))
    args = (o0, dev(probe), dev(inp.pos), dev(data), 4)
    r1 = P.cg_solve(*args, line_search=B)
    r2 = P.cg_solve(*args, line_search=B)
    assert torch.equal(r1.obj, r2.obj)
    assert r1.trace == r2.trace


def test_batched_needs_its_workspace(P):
    cfg, inp, probe, obj, data = workload("c1")
    d = P.dims_of(obj.shape, probe.shape[0], inp.pos.shape[0])
    small = P.workspace(d, torch.device("cuda"))
    with pytest.raises(P.PtygError) as e:
        P.cg_solve(dev(np.ones(obj.shape, np.complex64)), dev(probe), dev(inp.pos), dev(data), 2,
                   line_search=B, ws=small)
    assert e.value.status == -5


@pytest.mark.parametrize("case", ["m32", "m128"])
def test_batched_all_zero_intensities(P, case):
    """d = 0 everywhere: no element is listed for the per-trial pass (at
    n = 128 nothing is stored compacted) and every trial's objective comes
    from the zero-pixel polynomial."""
    cfg, inp, probe, obj, data = workload(case)
    zero = np.zeros_like(data)
    o0 = np.ones(obj.shape, np.complex64)
    res = P.cg_solve(dev(o0), dev(probe), dev(inp.pos), dev(zero), 3, line_search=B)
    ref, _ = cg_with_floor(o0, probe, inp.pos, zero, 3)
    print("zero data gammas", gammas(res.trace), gammas(ref[2]))
    assert gammas(res.trace) == gammas(ref[2])
    for a, b in zip(res.trace, ref[2]):
        assert abs(a["phi"] - b["phi"]) <= 1e-5 * abs(b["phi"])


def test_batched_nonfinite_data_is_reported(P):
    cfg, inp, probe, obj, data = workload("c1")
    bad = data.copy()
    bad[3, 2, 1] = np.nan
    with pytest.raises(P.PtygError) as e:
        P.cg_solve(dev(np.ones(obj.shape, np.complex64)), dev(probe), dev(inp.pos), dev(bad), 2, line_search=B)
    assert e.value.status == -4


def test_batched_workspace_sized_by_listed_count(P):
    """n = 128: a workspace sized by the data's listed-pixel count solves as
    the full one does; one pixel short is refused before anything is
    written past it."""
    cfg, inp, probe, obj, data = workload("m128")
    nnz = P.listed_count(dev(data), cfg.n)
    assert nnz == int(np.count_nonzero(~(data <= 0)))
    d = P.dims_of(obj.shape, cfg.n, cfg.k)
    args = (dev(np.ones(obj.shape, np.complex64)), dev(probe), dev(inp.pos), dev(data), 4)
    full = P.cg_solve(*args, line_search=B, ws=P.workspace(d, torch.device("cuda"), line_search=B), max_listed=-1)
    ws = P.workspace(d, torch.device("cuda"), line_search=B, max_listed=nnz)
    tight = P.cg_solve(*args, line_search=B, ws=ws, max_listed=nnz)
    assert torch.equal(full.obj, tight.obj) and full.trace == tight.trace
    short = P.workspace(d, torch.device("cuda"), line_search=B, max_listed=nnz - 1)
    with pytest.raises(P.PtygError) as e:
        P.cg_solve(*args, line_search=B, ws=short, max_listed=nnz - 1)
    assert e.value.status == -5
