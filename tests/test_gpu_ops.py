"""Parity of the HIP operators with the FP64 oracle (through the C ABI).

Tolerances: transforms are FP32 (unit roundoff 6e-8); a 2-D transform of
n^2 <= 65536 points adds O(log2 n^2) roundings, so per-operator relative L2
errors are ~1e-6.  The bound 1e-5 is the per-operator target; the forward
transform must also stay within twice the error of scipy's single-precision
FFT of the same exit waves (the same class of algorithm: radix-2/4 stages
with correctly rounded twiddles).  The gradient is held to the bound that
forward error implies through the residual's conditioning (_cases.grad_bound;
its residual and adjoint half alone is held to 1e-5 in test_gpu_grad_half).
Indexing (gather / scatter of integer-coded values) must be bit-exact."""
import numpy as np
import pytest

from oracle import ptycho as O

from _cases import grad_bound, rel, workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-5
CASES = ["c1", "m16r", "m32", "m64", "m128", "m256"]


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_07575_amd import ptyg
    ptyg.load()
    return ptyg


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_lane_swap_layout(P):
    a = torch.arange(64, dtype=torch.float32, device="cuda")
    b = 100 + torch.arange(64, dtype=torch.float32, device="cuda")
    P.debug_lane_swap(a, b)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(a[:32], np.arange(32)) and np.array_equal(a[32:], 100 + np.arange(32))
    assert np.array_equal(b[:32], 32 + np.arange(32)) and np.array_equal(b[32:], 100 + 32 + np.arange(32))


@pytest.mark.parametrize("n,h,w,k", [(16, 40, 57, 13), (32, 90, 70, 9), (64, 130, 100, 5), (128, 300, 260, 11),
                                     (256, 400, 300, 3)])
def test_gather_scatter_bit_exact(P, n, h, w, k):
    rng = np.random.default_rng(n)
    pos = np.stack([rng.integers(0, h - n + 1, k), rng.integers(0, w - n + 1, k)], 1).astype(np.int32)
    obj = np.add.outer(np.arange(h), 1j * np.arange(w)).astype(np.complex64)
    pat = P.debug_gather(dev(obj), dev(pos), n).cpu().numpy()
    assert np.array_equal(pat, O.gather(obj, pos, n))
    ipat = (rng.integers(-50, 50, (k, n, n)) + 1j * rng.integers(-50, 50, (k, n, n))).astype(np.complex64)
    out = P.debug_scatter(dev(ipat), dev(pos), (h, w)).cpu().numpy()
    assert np.array_equal(out, O.scatter_add(ipat.astype(np.complex128), pos, (h, w)).astype(np.complex64))


@pytest.mark.parametrize("case", CASES)
def test_forward_adjoint_parity(P, case):
    cfg, inp, probe, obj, data = workload(case)
    shape = obj.shape
    rng = np.random.default_rng(5)
    psi = (obj * (1 + 0.1 * rng.standard_normal(shape))).astype(np.complex64)
    far = P.forward(dev(psi), dev(probe), dev(inp.pos)).cpu().numpy()
    ref = O.forward(psi.astype(np.complex128), probe.astype(np.complex128), inp.pos)
    import scipy.fft
    n = probe.shape[0]
    sp32 = scipy.fft.fft2((probe[None] * O.gather(psi, inp.pos, n)).astype(np.complex64), norm="ortho")
    print(f"{case}: forward rel {rel(far, ref):.2e} (scipy float32 FFT {rel(sp32, ref):.2e})")
    assert rel(far, ref) <= TOL
    assert rel(far, ref) <= 2.0 * rel(sp32, ref)
    y = (rng.standard_normal(far.shape) + 1j * rng.standard_normal(far.shape)).astype(np.complex64)
    go, gp = P.adjoint(dev(y), dev(probe), dev(inp.pos), shape, obj=dev(psi), want_probe=True)
    ro, rp = O.adjoint(y.astype(np.complex128), probe.astype(np.complex128), inp.pos, shape,
                       obj=psi.astype(np.complex128))
    assert rel(go.cpu().numpy(), ro) <= TOL
    assert rel(gp.cpu().numpy(), rp) <= TOL
    # adjoint identity in FP32: <G x, y> = <x, G^H y>
    lhs = np.vdot(far.astype(np.complex128), y.astype(np.complex128))
    rhs = np.vdot(psi.astype(np.complex128), go.cpu().numpy().astype(np.complex128))
    assert abs(lhs - rhs) <= TOL * abs(lhs)


@pytest.mark.parametrize("case", ["c1", "m128", "m256"])
def test_normal_operator_illumination(P, case):
    cfg, inp, probe, obj, data = workload(case)
    far = P.forward(dev(obj), dev(probe), dev(inp.pos))
    ghg, _ = P.adjoint(far, dev(probe), dev(inp.pos), obj.shape)
    illum = O.illumination(probe.astype(np.complex128), inp.pos, obj.shape)
    assert rel(ghg.cpu().numpy(), illum * obj) <= TOL


@pytest.mark.parametrize("case", CASES)
def test_grad_and_objective_parity(P, case):
    cfg, inp, probe, obj, data = workload(case)
    rng = np.random.default_rng(7)
    for psi in [np.ones(obj.shape, np.complex64),
                (obj * (1 + 0.05 * rng.standard_normal(obj.shape))).astype(np.complex64)]:
        objective, g, gp = P.grad(dev(psi), dev(probe), dev(inp.pos), dev(data), want_probe=True)
        far = P.forward(dev(psi), dev(probe), dev(inp.pos)).cpu().numpy()
        ref, bo, bp, fo, fp = grad_bound(far, psi, probe, inp.pos, data, want_probe=True)
        phi, f = objective.cpu().numpy()
        eo, ep = rel(g.cpu().numpy(), ref["grad_obj"]), rel(gp.cpu().numpy(), ref["grad_probe"])
        print(f"{case}: phi rel {abs(phi - ref['phi']) / ref['phi']:.2e} grad_obj rel {eo:.2e} (bound {bo:.2e}, "
              f"fp32 floor {fo:.2e}) grad_probe rel {ep:.2e} (bound {bp:.2e}, floor {fp:.2e})")
        assert abs(phi - ref["phi"]) <= TOL * abs(ref["phi"])
        assert abs(f - ref["f"]) <= TOL * max(abs(ref["f"]), ref["phi"])
        assert eo <= bo
        assert ep <= bp


@pytest.mark.parametrize("case", CASES)
def test_minfunc_parity(P, case):
    cfg, inp, probe, obj, data = workload(case)
    rng = np.random.default_rng(9)
    psi = np.ones(obj.shape, np.complex64)
    eta = (0.1 * (rng.standard_normal(obj.shape) + 1j * rng.standard_normal(obj.shape))).astype(np.complex64)
    etap = (0.01 * np.abs(probe).max() * (rng.standard_normal(probe.shape))).astype(np.complex64)
    for gamma in [0.0, 0.5, 0.0625]:
        for with_p in [False, True]:
            val = P.minfunc(dev(psi), dev(probe), dev(inp.pos), dev(data), dir_obj=dev(eta),
                            dir_probe=dev(etap) if with_p else None, gamma=gamma).cpu().numpy()
            g32 = np.float32(gamma)
            oo = (psi + g32 * eta).astype(np.complex128)
            pp = (probe + g32 * etap).astype(np.complex128) if with_p else probe.astype(np.complex128)
            phi, f = O.minfunc(oo, pp, inp.pos, data.astype(np.float64))
            assert abs(val[0] - phi) <= TOL * abs(phi)


def test_position_check(P):
    cfg, inp, probe, obj, data = workload("c1")
    P.check_positions(dev(inp.pos), obj.shape, 16)
    bad = inp.pos.copy()
    bad[3] = (obj.shape[0] - 15, 0)
    with pytest.raises(P.PtygError) as e:
        P.check_positions(dev(bad), obj.shape, 16)
    assert e.value.status == -2
    with pytest.raises(ValueError):
        P.positions(torch.tensor([[1.5, 2.0]]))


def test_grad_and_adjoint_are_bit_reproducible(P):
    cfg, inp, probe, obj, data = workload("m128")
    psi = dev(obj)
    a = P.grad(psi, dev(probe), dev(inp.pos), dev(data), want_probe=True)
    b = P.grad(psi, dev(probe), dev(inp.pos), dev(data), want_probe=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
