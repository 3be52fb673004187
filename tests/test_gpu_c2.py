"""Full-size single-projection workload (2048^2 object, 128^2 probe, 4096
positions, Poisson at 1e5 photons) in the launch configuration the benchmark
times: the linear operators, the residual and adjoint half of GRAD, the full
GRAD and a CG iteration against the oracle at full size."""
import numpy as np
import pytest

from oracle import ptycho as O

from _cases import grad_bound, rel, workload
from _gpu import dev, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-5


@pytest.fixture(scope="module")
def P():
    return lib()


def test_c2_linear_operators_full_size(P):
    cfg, inp, probe, obj, data = workload("c2")
    p64 = probe.astype(np.complex128)
    far = P.forward(dev(obj), dev(probe), dev(inp.pos))
    ref = O.forward(obj.astype(np.complex128), p64, inp.pos)
    ef = rel(far.cpu().numpy(), ref)
    del ref
    # G^H G = illumination (unitary F)
    ghg, _ = P.adjoint(far, dev(probe), dev(inp.pos), obj.shape)
    del far
    illum = O.illumination(p64, inp.pos, obj.shape)
    en = rel(ghg.cpu().numpy(), illum * obj)
    # adjoint of a seeded random far field
    rng = np.random.default_rng(21)
    y = (rng.standard_normal((cfg.k, cfg.n, cfg.n), np.float32)
         + 1j * rng.standard_normal((cfg.k, cfg.n, cfg.n), np.float32)).astype(np.complex64)
    go, _ = P.adjoint(dev(y), dev(probe), dev(inp.pos), obj.shape)
    ro, _ = O.adjoint(y.astype(np.complex128), p64, inp.pos, obj.shape)
    ea = rel(go.cpu().numpy(), ro)
    print(f"c2 full size: forward rel {ef:.2e}, G^H G vs illumination rel {en:.2e}, adjoint rel {ea:.2e}")
    assert ef <= TOL and en <= TOL and ea <= TOL


def test_c2_grad_half_full_size(P):
    cfg, inp, probe, obj, data = workload("c2")
    psi = np.ones(obj.shape, np.complex64)
    p64 = probe.astype(np.complex128)
    d64 = data.astype(np.float64)
    g32 = O.forward(psi.astype(np.complex128), p64, inp.pos).astype(np.complex64)
    objective, go, _, _ = P.debug_grad_far(dev(g32), dev(probe), dev(inp.pos), dev(data), obj.shape)
    g = g32.astype(np.complex128)
    ro, _ = O.adjoint(O.residual(g, d64), p64, inp.pos, obj.shape)
    _, dterms = O.objective_terms(np.abs(g) ** 2, d64)
    eo = rel(go.cpu().numpy(), ro)
    phi_ref = float(np.sum(dterms))
    print(f"c2 residual + adjoint half on the oracle's far field: grad rel {eo:.2e}, "
          f"phi rel {abs(objective[0].item() - phi_ref) / phi_ref:.2e}")
    assert eo <= TOL
    assert abs(objective[0].item() - phi_ref) <= TOL * phi_ref


def test_c2_grad_full_size(P):
    cfg, inp, probe, obj, data = workload("c2")
    psi = np.ones(obj.shape, np.complex64)
    objective, g, _ = P.grad(dev(psi), dev(probe), dev(inp.pos), dev(data))
    far = P.forward(dev(psi), dev(probe), dev(inp.pos)).cpu().numpy()
    ref, bo, _, fo, _ = grad_bound(far, psi, probe, inp.pos, data)
    phi, f = objective.cpu().numpy()
    eo = rel(g.cpu().numpy(), ref["grad_obj"])
    print(f"c2 phi gpu {phi:.10e} oracle {ref['phi']:.10e}; grad rel {eo:.2e} (bound {bo:.2e}, fp32 floor {fo:.2e})")
    assert abs(phi - ref["phi"]) <= TOL * ref["phi"]
    assert abs(f - ref["f"]) <= TOL * max(abs(ref["f"]), ref["phi"])
    assert eo <= bo
