"""The residual and adjoint half of GRAD (Eqs. ML and gradient) on a given
far field, against the oracle on the same far field.

ptyg_debug_grad_far runs GRAD's own residual / objective epilogue, inverse
transform, overlap sum (and probe-gradient reduction) on a far field the
caller supplies.  It is fed the oracle's far field g = G psi rounded once to
FP32, and compared with the oracle's gradient of that same rounded far
field, G^H r(g32): no far-field error enters, so nothing is amplified by the
residual's conditioning and the per-operator bound 1e-5 applies to the
gradients and objectives.  The residual itself is checked element by
element where |g|^2 >= eps: forming 1 - d / |g|^2 with an approximate
reciprocal and scaling g by it costs a few roundings of |g| (1 + d / |g|^2),
so |r_gpu - r| <= 8 u |g| (1 + d / |g|^2) with u = 2^-24 (Poisson), and
|g| (1 + sqrt(d) / |g|) in place of |g| (1 + d / |g|^2) for least squares."""
import numpy as np
import pytest

from oracle import ptycho as O

from _cases import rel, workload
from _gpu import dev, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-5
U = 2.0 ** -24


@pytest.fixture(scope="module")
def P():
    return lib()


def check_half(P, psi, probe, pos, data, want_probe, estimator="ml", label=""):
    p64 = probe.astype(np.complex128)
    psi64 = psi.astype(np.complex128)
    d64 = data.astype(np.float64)
    g32 = O.forward(psi64, p64, pos).astype(np.complex64)
    g = g32.astype(np.complex128)
    objective, go, gp, res = P.debug_grad_far(dev(g32), dev(probe), dev(pos), dev(data), psi.shape, obj=dev(psi),
                                              want_probe=want_probe, estimator=estimator)
    r = O.residual(g, d64, estimator=estimator)
    ro, rp = O.adjoint(r, p64, pos, psi.shape, obj=psi64 if want_probe else None)
    paper, dev_terms = O.objective_terms(np.abs(g) ** 2, d64, estimator=estimator)
    phi_ref, f_ref = float(np.sum(dev_terms)), float(np.sum(paper))
    phi, f = objective.cpu().numpy()
    eo = rel(go.cpu().numpy(), ro)
    x = np.abs(g) ** 2
    big = x >= O.EPS
    if estimator == "ls":
        cond = np.abs(g) + np.sqrt(np.maximum(d64, 0.0))
    else:
        cond = np.abs(g) * (1.0 + d64 / np.where(big, x, 1.0))
    rerr = np.abs(res.cpu().numpy().astype(np.complex128) - r)
    worst = float(np.max(np.where(big, rerr / np.maximum(8 * U * cond, 1e-300), 0.0)))
    msg = (f"{label}: grad_obj rel {eo:.2e}, phi rel {abs(phi - phi_ref) / max(abs(phi_ref), 1e-300):.2e}, "
           f"residual worst / bound {worst:.3f}")
    if want_probe:
        ep = rel(gp.cpu().numpy(), rp)
        msg += f", grad_probe rel {ep:.2e}"
    print(msg)
    assert eo <= TOL
    assert abs(phi - phi_ref) <= TOL * max(abs(phi_ref), 1e-300)
    assert abs(f - f_ref) <= TOL * max(abs(f_ref), abs(phi_ref))
    assert worst <= 1.0
    if want_probe:
        assert ep <= TOL


@pytest.mark.parametrize("case", ["c1", "m16r", "m32", "m64", "m128", "m256"])
@pytest.mark.parametrize("want_probe", [False, True])
def test_grad_half_on_oracle_far_field(P, case, want_probe):
    cfg, inp, probe, obj, data = workload(case)
    rng = np.random.default_rng(11)
    for i, psi in enumerate([np.ones(obj.shape, np.complex64),
                             (obj * (1 + 0.05 * rng.standard_normal(obj.shape))).astype(np.complex64)]):
        check_half(P, psi, probe, inp.pos, data, want_probe, label=f"{case} psi{i} probe={want_probe}")


@pytest.mark.parametrize("case", ["m32", "m128", "m256"])
def test_grad_half_least_squares(P, case):
    cfg, inp, probe, obj, data = workload(case)
    check_half(P, np.ones(obj.shape, np.complex64), probe, inp.pos, data, True, estimator="ls",
               label=f"{case} least squares")


def test_grad_half_zero_far_field_is_guarded(P):
    # g = 0 everywhere: x < eps, so r = g = 0 and the gradient is exactly 0;
    # the objective is sum over d > 0 of d (1 - log(eps / d)) ... as the oracle forms it
    cfg, inp, probe, obj, data = workload("m32")
    g32 = np.zeros((cfg.k, cfg.n, cfg.n), np.complex64)
    objective, go, _, res = P.debug_grad_far(dev(g32), dev(probe), dev(inp.pos), dev(data), obj.shape)
    assert not torch.any(go != 0) and not torch.any(res != 0)
    paper, dev_terms = O.objective_terms(np.zeros(data.shape), data.astype(np.float64))
    assert abs(objective[0].item() - np.sum(dev_terms)) <= TOL * np.sum(dev_terms)
