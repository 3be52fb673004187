"""Pins of the oracle's least-squares estimator (the LS estimate the paper
names in section Background without a formula; read as
F = sum (|g| - sqrt d)^2, gradient G^H (g - sqrt(d) g / |g|) in the
Wirtinger convention of Eq. gradient)."""
import numpy as np
import pytest

from oracle import ptycho as O
from paper_2106_07575_amd import synth


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture(scope="module")
def c1():
    cfg = synth.CONFIGS["c1"]
    inp = synth.make_inputs(cfg)
    d = synth.make_data(cfg, np.abs(O.forward(inp.obj_true, inp.probe, inp.pos)) ** 2)
    return cfg, inp, d


def test_hand_values():
    # g = 3 + 4i (|g| = 5): d = 16 -> (5 - 4)^2 = 1, r = g (1 - 4/5) = 0.6 + 0.8i;
    # d = 25 -> 0 and r = 0; d = 0 -> |g|^2 = 25 and r = g
    g = np.array([3 + 4j, 3 + 4j, 3 + 4j])
    d = np.array([16.0, 25.0, 0.0])
    paper, dev = O.objective_terms(np.abs(g) ** 2, d, estimator="ls")
    assert np.array_equal(paper, dev)
    assert paper == pytest.approx([1.0, 0.0, 25.0], abs=1e-14)
    r = O.residual(g, d, estimator="ls")
    assert r == pytest.approx([0.6 + 0.8j, 0.0, 3 + 4j], abs=1e-14)
    # below the guard the residual is g itself
    assert O.residual(np.array([1e-20 + 0j]), np.array([4.0]), estimator="ls")[0] == 1e-20


def test_zero_data_matches_ml():
    """d = 0: both estimators are sum |G psi|^2 with gradient G^H G psi."""
    h, w, n = 40, 36, 8
    rng = np.random.default_rng(5)
    pos = np.stack([rng.integers(0, h - n + 1, 11), rng.integers(0, w - n + 1, 11)], 1)
    psi, p = _rand((h, w), 1), _rand((n, n), 2)
    d = np.zeros((11, n, n))
    a = O.grad(psi, p, pos, d, want_probe=True, estimator="ls")
    b = O.grad(psi, p, pos, d, want_probe=True, estimator="ml")
    assert a["phi"] == pytest.approx(b["phi"], rel=1e-14)
    assert np.allclose(a["grad_obj"], b["grad_obj"], rtol=0, atol=1e-12)
    assert np.allclose(a["grad_probe"], b["grad_probe"], rtol=0, atol=1e-12)


def test_zero_gradient_and_objective_at_truth(c1):
    cfg, inp, d = c1
    res = O.grad(inp.obj_true, inp.probe, inp.pos, d, estimator="ls")
    res0 = O.grad(synth.initial_object(cfg), inp.probe, inp.pos, d, estimator="ls")
    assert abs(res["phi"]) <= 1e-12 * res0["phi"]
    assert np.linalg.norm(res["grad_obj"]) <= 1e-10 * np.linalg.norm(res0["grad_obj"])


def test_finite_difference_gradient_object_and_probe(c1):
    cfg, inp, d = c1
    psi = synth.initial_object(cfg) * 0.95 + 0.05 * inp.obj_true
    p = inp.probe * 1.1
    res = O.grad(psi, p, inp.pos, d, want_probe=True, estimator="ls")
    for seed in range(3):
        v = _rand(psi.shape, 100 + seed)
        v *= np.linalg.norm(psi) / np.linalg.norm(v)
        h = 1e-6
        fd = (O.minfunc(psi + h * v, p, inp.pos, d, estimator="ls")[1]
              - O.minfunc(psi - h * v, p, inp.pos, d, estimator="ls")[1]) / (2 * h)
        an = 2 * np.vdot(res["grad_obj"], v).real
        assert abs(fd - an) <= 1e-6 * abs(an)
        q = _rand(p.shape, 200 + seed)
        q *= np.linalg.norm(p) / np.linalg.norm(q)
        fd = (O.minfunc(psi, p + h * q, inp.pos, d, estimator="ls")[1]
              - O.minfunc(psi, p - h * q, inp.pos, d, estimator="ls")[1]) / (2 * h)
        an = 2 * np.vdot(res["grad_probe"], q).real
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_ls_cg_descends_toward_truth(c1):
    cfg, inp, d = c1
    psi0 = synth.initial_object(cfg)
    obj, _, tr = O.cg_solve(psi0, inp.probe, inp.pos, d, 16, estimator="ls")
    phis = [r["phi"] for r in tr]
    assert all(b <= a for a, b in zip(phis, phis[1:]))
    illum = O.illumination(inp.probe, inp.pos, psi0.shape)
    mask = illum >= 1e-3 * illum.max()
    e0 = np.linalg.norm(O.align_phase(psi0, inp.obj_true, mask)[mask] - inp.obj_true[mask])
    e1 = np.linalg.norm(O.align_phase(obj, inp.obj_true, mask)[mask] - inp.obj_true[mask])
    assert e1 < 0.5 * e0
