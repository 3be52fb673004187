"""Boundary and degenerate cases of the operator and the solver against the
oracle (Eqs. fwd_model, ML, gradient; Algorithm 1):

* one pattern on an object no larger than the probe (the only position is
  the origin), and two patterns at opposite corners of a ragged object (the
  last valid position on both axes), for every probe size: forward and
  adjoint (object and probe) at 1e-5, Phi at 1e-5, the object and probe
  gradients within the bound of _cases.grad_bound;
* zero CG iterations in both line-search modes: nothing changes, no trace;
* solves on host threads that end (each frees its pinned readback buffer)
  give the same iterates as on the test's own thread."""
import numpy as np
import pytest

from oracle import ptycho as O
from paper_2106_07575_amd import synth

from _cases import grad_bound, rel
from _gpu import dev, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-5


@pytest.fixture(scope="module")
def P():
    return lib()


def case(n, h, w, pos, seed):
    rng = np.random.default_rng(seed)
    probe = synth.make_probe(n, "disk", 1e4, seed).astype(np.complex64)
    obj = (np.exp(1j * 0.3 * rng.standard_normal((h, w))) * rng.uniform(0.9, 1.0, (h, w))).astype(np.complex64)
    pos = np.asarray(pos, np.int32)
    inten = np.abs(O.forward(obj.astype(np.complex128), probe.astype(np.complex128), pos)) ** 2
    data = synth.poisson_counts(inten, seed + 1)
    return probe, obj, pos, data


def check(P, probe, obj, pos, data, label):
    p64, o64 = probe.astype(np.complex128), obj.astype(np.complex128)
    far = P.forward(dev(obj), dev(probe), dev(pos))
    ref_far = O.forward(o64, p64, pos)
    ef = rel(far.cpu().numpy(), ref_far)
    y = ref_far.astype(np.complex64)
    go, gp = P.adjoint(dev(y), dev(probe), dev(pos), obj.shape, obj=dev(obj), want_probe=True)
    ro, rp = O.adjoint(y.astype(np.complex128), p64, pos, obj.shape, obj=o64)
    ea, ep = rel(go.cpu().numpy(), ro), rel(gp.cpu().numpy(), rp)
    objective, g, gpr = P.grad(dev(obj), dev(probe), dev(pos), dev(data), want_probe=True)
    ref, bo, bp, _, _ = grad_bound(far.cpu().numpy(), obj, probe, pos, data, want_probe=True)
    ephi = abs(objective[0].item() - ref["phi"]) / ref["phi"]
    eg, egp = rel(g.cpu().numpy(), ref["grad_obj"]), rel(gpr.cpu().numpy(), ref["grad_probe"])
    print(f"{label}: forward {ef:.1e}, adjoint {ea:.1e} / {ep:.1e}, phi {ephi:.1e}, grad {eg:.1e} (bound {bo:.1e}), "
          f"probe grad {egp:.1e} (bound {bp:.1e})")
    assert ef <= TOL and ea <= TOL and ep <= TOL and ephi <= TOL
    assert eg <= bo and egp <= bp


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256])
def test_one_pattern_object_the_size_of_the_probe(P, n):
    probe, obj, pos, data = case(n, n, n, [[0, 0]], 300 + n)
    check(P, probe, obj, pos, data, f"n={n}, one pattern, {n}x{n} object")


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256])
def test_two_patterns_at_opposite_corners(P, n):
    h, w = n + 37, n + 19
    probe, obj, pos, data = case(n, h, w, [[0, 0], [h - n, w - n]], 400 + n)
    check(P, probe, obj, pos, data, f"n={n}, corners of {h}x{w}")


@pytest.mark.parametrize("ls", ["sequential", "batched"])
def test_zero_iterations_change_nothing(P, ls):
    probe, obj, pos, data = case(32, 80, 70, [[0, 0], [20, 10], [48, 38]], 500)
    psi = np.ones(obj.shape, np.complex64)
    res = P.cg_solve(dev(psi), dev(probe), dev(pos), dev(data), 0, update_probe=True, line_search=ls)
    assert res.iters_done == 0 and res.trace == []
    assert np.array_equal(res.obj.cpu().numpy(), psi) and np.array_equal(res.probe.cpu().numpy(), probe)


@pytest.mark.parametrize("ls", ["sequential", "batched"])
def test_solves_on_threads_that_end(P, ls):
    # each host thread owns a pinned readback buffer, freed when the thread
    # ends: solves on short-lived threads match the same solve on this one
    import threading

    probe, obj, pos, data = case(32, 80, 70, [[0, 0], [20, 10], [48, 38]], 510)
    args = lambda: (dev(np.ones(obj.shape, np.complex64)), dev(probe), dev(pos), dev(data), 3)
    ref = P.cg_solve(*args(), line_search=ls)
    for _ in range(3):
        out = {}
        th = threading.Thread(target=lambda: out.update(r=P.cg_solve(*args(), line_search=ls)))
        th.start()
        th.join()
        r = out["r"]
        assert [t["phi"] for t in r.trace] == [t["phi"] for t in ref.trace]
        assert np.array_equal(r.obj.cpu().numpy(), ref.obj.cpu().numpy())
