"""torch.autograd wrappers (differentiable operator, joint object+probe
gradient) on the c3 workload: 1024^2 object and 128^2 probe as leaves, 2048
uniform positions, Poisson data at 1e4 photons.  Checked by central finite
differences (64 seeded directions, each a random unit vector plus the unit
gradient, scaled to ||v|| = ||x||) and against the oracle gradient.  The
step is h = 1e-6: the Poisson log term is nearly singular at dim far-field
pixels with counts, and along such directions the FP64 oracle's own central
difference is off by 1.6e-2 at h = 1e-5 and 1.1e-4 at h = 1e-6 (O(h^2));
at h = 1e-3 it is off by up to 40% even along random directions."""
import numpy as np
import pytest

from oracle import ptycho as O

from _cases import grad_tol, grad_with_floor, rel, workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_07575_amd import autograd as AG
    from paper_2106_07575_amd import ptyg
    cfg, inp, probe, obj, data = workload("c3")
    rng = np.random.default_rng(33)
    psi = (obj * (1 + 0.1 * (rng.standard_normal(obj.shape) + 1j * rng.standard_normal(obj.shape)))
           ).astype(np.complex64)
    p = (probe * (1 + 0.05 * rng.standard_normal(probe.shape))).astype(np.complex64)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return AG, ptyg, dev, inp, psi, p, data


def test_ml_loss_finite_differences_joint(env):
    AG, ptyg, dev, inp, psi, p, data = env
    pos, d = dev(inp.pos), dev(data)
    o = dev(psi).requires_grad_(True)
    q = dev(p).requires_grad_(True)
    loss = AG.ml_loss(o, q, pos, d)
    loss.backward()
    go, gq = o.grad, q.grad
    assert loss.dtype == torch.float64
    gen = torch.Generator(device="cuda").manual_seed(5)
    gnorm = torch.sqrt(torch.linalg.vector_norm(go) ** 2 + torch.linalg.vector_norm(gq) ** 2)
    h = 1e-6
    errs = []
    with torch.no_grad():
        for j in range(64):
            # random direction plus the gradient direction: a purely random
            # direction in 2.1M real dimensions is nearly orthogonal to the
            # gradient, and its tiny derivative drowns in FP32 loss noise
            vo = torch.randn(o.shape, dtype=torch.complex64, device="cuda", generator=gen)
            vq = torch.randn(q.shape, dtype=torch.complex64, device="cuda", generator=gen)
            vo = vo / torch.linalg.vector_norm(vo) + go / gnorm
            vq = vq / torch.linalg.vector_norm(vq) + gq / gnorm
            vo *= torch.linalg.vector_norm(o) / torch.linalg.vector_norm(vo)
            vq *= torch.linalg.vector_norm(q) / torch.linalg.vector_norm(vq)
            lp = AG.ml_loss(o + h * vo, q + h * vq, pos, d).item()
            lm = AG.ml_loss(o - h * vo, q - h * vq, pos, d).item()
            fd = (lp - lm) / (2 * h)
            # torch convention: dL = Re <grad, dz> summed over leaves
            an = (torch.vdot(go.flatten().to(torch.complex128), vo.flatten().to(torch.complex128)).real
                  + torch.vdot(gq.flatten().to(torch.complex128), vq.flatten().to(torch.complex128)).real).item()
            errs.append(abs(fd - an) / abs(an))
    print(f"FD over 64 directions: max rel {max(errs):.2e}, median {np.median(errs):.2e}")
    assert max(errs) <= 1e-3


def test_ml_loss_gradient_matches_oracle(env):
    AG, ptyg, dev, inp, psi, p, data = env
    o = dev(psi).requires_grad_(True)
    q = dev(p).requires_grad_(True)
    loss = AG.ml_loss(o, q, dev(inp.pos), dev(data))
    loss.backward()
    ref, fo, fp = grad_with_floor(psi, p, inp.pos, data, want_probe=True)
    assert abs(loss.item() - ref["phi"]) <= 1e-5 * ref["phi"]
    eo = rel(o.grad.cpu().numpy(), 2 * ref["grad_obj"])
    ep = rel(q.grad.cpu().numpy(), 2 * ref["grad_probe"])
    print(f"autograd vs 2x oracle gradient: object {eo:.2e} (floor {fo:.2e}), probe {ep:.2e} (floor {fp:.2e})")
    assert eo <= grad_tol(fo) and ep <= grad_tol(fp)
    # Eq. ML form: same gradient, value F
    o2 = dev(psi).requires_grad_(True)
    l2 = AG.ml_loss(o2, dev(p), dev(inp.pos), dev(data), which="eq_ml")
    l2.backward()
    assert abs(l2.item() - ref["f"]) <= 1e-5 * max(abs(ref["f"]), ref["phi"])
    assert rel(o2.grad.cpu().numpy(), o.grad.cpu().numpy()) <= 1e-6


def test_far_field_vjp_is_the_adjoint(env):
    AG, ptyg, dev, inp, psi, p, data = env
    pos = dev(inp.pos)
    o = dev(psi).requires_grad_(True)
    q = dev(p).requires_grad_(True)
    far = AG.far_field(o, q, pos)
    gen = torch.Generator(device="cuda").manual_seed(9)
    w = torch.randn(far.shape, dtype=torch.complex64, device="cuda", generator=gen)
    # L = Re <w, far> is linear: its finite difference is exact up to rounding
    L = torch.vdot(w.flatten(), far.flatten()).real
    L.backward()
    with torch.no_grad():
        for j in range(4):
            vo = torch.randn(o.shape, dtype=torch.complex64, device="cuda", generator=gen)
            fo = torch.vdot(w.flatten(), ptyg.forward(vo, q, pos).flatten()).real.item()
            an = torch.vdot(o.grad.flatten(), vo.flatten()).real.item()
            assert abs(fo - an) <= 1e-5 * abs(fo)
            vq = torch.randn(q.shape, dtype=torch.complex64, device="cuda", generator=gen)
            fq = torch.vdot(w.flatten(), ptyg.forward(o.detach(), vq, pos).flatten()).real.item()
            an = torch.vdot(q.grad.flatten(), vq.flatten()).real.item()
            assert abs(fq - an) <= 1e-5 * abs(fq)
    # against the oracle adjoint
    ro, rp = O.adjoint(w.cpu().numpy().astype(np.complex128), p.astype(np.complex128), inp.pos, psi.shape,
                       obj=psi.astype(np.complex128))
    assert rel(o.grad.cpu().numpy(), ro) <= 1e-5
    assert rel(q.grad.cpu().numpy(), rp) <= 1e-5


def test_far_field_composes_with_torch_loss(env):
    AG, ptyg, dev, inp, psi, p, data = env
    o = dev(psi).requires_grad_(True)
    far = AG.far_field(o, dev(p), dev(inp.pos))
    L = (far.abs() ** 2).sum()          # = sum |G psi|^2 ; dL/d conj(psi) = G^H G psi
    L.backward()
    illum = O.illumination(p.astype(np.complex128), inp.pos, psi.shape)
    assert rel(o.grad.cpu().numpy(), 2 * illum * psi) <= 1e-5
