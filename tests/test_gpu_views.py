"""Multi-view batch (ptyg_cg_solve_views): V independent projections in one
set of launches must give, view by view, what the oracle's CG gives for each
view alone -- identical line-search decisions on the well-conditioned
32^2 workload (also with a pattern count per view that the batch pads), the
iterate bound of _cases.trajectory_factor on the 128^2 one."""
import numpy as np
import pytest

from oracle import ptycho as O

from _cases import cg_with_floor, rel, views_workload
from _gpu import start_factors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_07575_amd import ptyg
    ptyg.load()
    return ptyg


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("ls", ["batched", "sequential"])
def test_views_exact_decisions_32(P, ls):
    probe, objs, pos, data = views_workload(32, 3)
    V = objs.shape[0]
    obj0 = np.ones(objs.shape, np.complex64)
    print(f"views 32 x{V} {ls}", flush=True)
    out, traces, done = P.cg_solve_views(dev(obj0), dev(probe), dev(pos), dev(data), 8, line_search=ls)
    assert done == 8
    for v in range(V):
        (ro, rp, rtr), _ = cg_with_floor(obj0[v], probe, pos[v], data[v], 8)
        err = rel(out[v].cpu().numpy(), ro)
        print(f"   view {v}: object rel {err:.2e}", [r["gamma"] for r in traces[v]])
        assert [r["gamma"] for r in traces[v]] == [r["gamma"] for r in rtr]
        assert [r["halvings"] for r in traces[v]] == [r["halvings"] for r in rtr]
        for a, b in zip(traces[v], rtr):
            assert abs(a["phi"] - b["phi"]) <= 1e-5 * abs(b["phi"])
        assert err <= 1e-3


def test_views_within_fp32_floor_128(P):
    probe, objs, pos, data = views_workload(128, 2)
    V = objs.shape[0]
    obj0 = np.ones(objs.shape, np.complex64)
    out, traces, done = P.cg_solve_views(dev(obj0), dev(probe), dev(pos), dev(data), 4)
    for v in range(V):
        (ro, rp, rtr), (po, pp, ptr) = cg_with_floor(obj0[v], probe, pos[v], data[v], 4)
        illum = O.illumination(probe.astype(np.complex128), pos[v], objs.shape[1:])
        mask = illum >= 1e-3 * illum.max()
        err, floor = rel(out[v].cpu().numpy()[mask], ro[mask]), rel(po[mask], ro[mask])
        print(f"views 128 view {v}: object rel {err:.2e} (floor {floor:.2e})")
        c, _ = start_factors(P, obj0[v], probe, pos[v], data[v])
        assert err <= max(1e-3, c * floor)
        assert traces[v][0]["gamma"] == rtr[0]["gamma"]


def test_single_view_matches_cg_solve(P):
    probe, objs, pos, data = views_workload(32, 3)
    o0 = np.ones(objs.shape[1:], np.complex64)
    a = P.cg_solve(dev(o0), dev(probe), dev(pos[1]), dev(data[1]), 6, line_search="batched")
    out, traces, _ = P.cg_solve_views(dev(o0[None]), dev(probe), dev(pos[1:2]), dev(data[1:2]), 6)
    assert [r["gamma"] for r in a.trace] == [r["gamma"] for r in traces[0]]
    assert rel(out[0].cpu().numpy(), a.obj.cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("ls", ["batched", "sequential"])
@pytest.mark.parametrize("k", [61, 63])
def test_views_ragged_pattern_count(P, ls, k):
    # k not a multiple of the 8 patterns per workgroup at n = 32: each view is
    # padded with patterns on zero rows below the stacked views, which must
    # change nothing -- the oracle's decisions for every view alone, and the
    # caller's object gets the iterates back
    probe, objs, pos, data = views_workload(32, 3)
    pos, data = pos[:, :k], data[:, :k]
    V = objs.shape[0]
    obj0 = np.ones(objs.shape, np.complex64)
    print(f"views 32 x{V}, k = {k}, {ls}", flush=True)
    out, traces, done = P.cg_solve_views(dev(obj0), dev(probe), dev(pos), dev(data), 6, line_search=ls)
    assert done == 6
    for v in range(V):
        (ro, rp, rtr), _ = cg_with_floor(obj0[v], probe, pos[v], data[v], 6)
        err = rel(out[v].cpu().numpy(), ro)
        print(f"   view {v}: object rel {err:.2e}", [r["halvings"] for r in traces[v]])
        assert [r["halvings"] for r in traces[v]] == [r["halvings"] for r in rtr]
        for a, b in zip(traces[v], rtr):
            assert abs(a["phi"] - b["phi"]) <= 1e-5 * abs(b["phi"])
        assert err <= 1e-3


def test_views_argument_errors(P):
    probe, objs, pos, data = views_workload(32, 3)
    o0 = np.ones(objs.shape, np.complex64)
    with pytest.raises(P.PtygError) as e:
        P.cg_solve_views(dev(o0), dev(probe), dev(pos), dev(data), 2, max_halvings=0)
    assert e.value.status == -1
    bad = pos.copy()
    bad[2, 5] = (objs.shape[1] - 31, 0)
    with pytest.raises(P.PtygError) as e:
        P.cg_solve_views(dev(o0), dev(probe), dev(bad), dev(data), 2)
    assert e.value.status == -2
