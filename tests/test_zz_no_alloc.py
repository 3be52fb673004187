"""ptyg_minfunc_noalloc (no workspace, partials in the library's fixed device
array) against ptyg_minfunc (caller workspace) through the C ABI: the same
kernels and reduction, so the objectives must agree bit for bit; two calls
in a row, the second on a smaller input, so the array is reused."""
import numpy as np
import pytest

from oracle import ptycho as O

from _cases import workload
from _gpu import dev, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    return lib()


def test_minfunc_noalloc_matches_workspace_call(P):
    rng = np.random.default_rng(17)
    for case, k in [("m128", None), ("m32", 20)]:
        cfg, inp, probe, obj, data = workload(case)
        pos, d = inp.pos, data
        if k is not None:
            pos, d = pos[:k], data[:k]
        psi = np.ones(obj.shape, np.complex64)
        eta = (0.1 * (rng.standard_normal(obj.shape) + 1j * rng.standard_normal(obj.shape))).astype(np.complex64)
        out = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
        P.minfunc_noalloc(dev(psi), dev(probe), dev(pos), dev(d), out, dir_obj=dev(eta), gamma=0.25)
        ref = P.minfunc(dev(psi), dev(probe), dev(pos), dev(d), dir_obj=dev(eta), gamma=0.25)
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        phi_o, f_o = O.minfunc((psi + np.float32(0.25) * eta).astype(np.complex128), probe.astype(np.complex128),
                               pos, d.astype(np.float64))
        print(f"{case} k={len(pos)}: noalloc {got}, workspace call {want}, oracle {phi_o:.10e}")
        assert np.array_equal(got, want)
        assert abs(got[0] - phi_o) <= 1e-5 * phi_o


def test_minfunc_noalloc_rejects_oversize(P):
    cfg, inp, probe, obj, data = workload("m256")
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PtygError) as e:
        P.minfunc_noalloc(dev(np.ones(obj.shape, np.complex64)), dev(probe), dev(inp.pos), dev(data), out)
    assert e.value.status == -1


def test_minfunc_noalloc_rejects_too_many_patterns(P):
    # k beyond the array's rows is refused from the dims alone, before any
    # launch (the small buffers are never read)
    import ctypes
    d = P.Dims(256, 256, 128, 70000)
    buf = torch.zeros(1024, dtype=torch.float64, device="cuda")
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    st = P.load().ptyg_minfunc_noalloc(ctypes.byref(d), P._ptr(buf), None, P._ptr(buf), None, 0.0, P._ptr(buf),
                                       P._ptr(buf), 1e-32, 0, P._ptr(out), P._stream())
    assert st == -1
    assert "65536" in P.load().ptyg_last_error().decode()
