"""Pins of the oracle's objective, residual and gradients (Eq. ML, Eq. gradient)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ptycho as O
from paper_2106_07575_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture(scope="module")
def c1():
    cfg = synth.CONFIGS["c1"]
    inp = synth.make_inputs(cfg)
    d = synth.make_data(cfg, np.abs(O.forward(inp.obj_true, inp.probe, inp.pos)) ** 2)
    return cfg, inp, d


def test_hand_fixture_objective_and_gradients():
    g = json.load(open(os.path.join(GOLD, "hand_2x2.json")))
    obj = np.array(g["obj_re"], complex)
    probe = np.array(g["probe_re"]) + 1j * np.array(g["probe_im"])
    pos = np.array(g["pos"], np.int32)
    d = np.array(g["data"], float)
    res = O.grad(obj, probe, pos, d, want_probe=True)
    assert res["phi"] == pytest.approx(g["objective_deviance"], rel=1e-14)
    assert res["f"] == pytest.approx(g["objective_paper"], rel=1e-14)
    go = np.array(g["grad_obj_re"]) + 1j * np.array(g["grad_obj_im"])
    gp = np.array(g["grad_probe_re"]) + 1j * np.array(g["grad_probe_im"])
    assert np.allclose(res["grad_obj"], go, atol=1e-13)
    assert np.allclose(res["grad_probe"], gp, atol=1e-13)
    phi, f = O.minfunc(obj, probe, pos, d)
    assert phi == pytest.approx(res["phi"], rel=1e-15) and f == pytest.approx(res["f"], rel=1e-15)


def test_objective_terms_closed_forms():
    x = np.array([2.0, 1.0, 0.0, 3.0, 5.0])
    d = np.array([1.0, 1.0, 0.0, 0.0, 2.0])
    paper, dev = O.objective_terms(x, d)
    assert paper[0] == pytest.approx(2 - math.log(2), rel=1e-15)
    assert dev[0] == pytest.approx(1 - math.log(2), rel=1e-15)
    assert dev[1] == 0.0 and paper[1] == 1.0
    assert paper[2] == 0.0 and dev[2] == 0.0
    assert paper[3] == 3.0 and dev[3] == 3.0
    # dev = paper - (d - d log d) where d > 0
    assert dev[4] == pytest.approx(paper[4] - (2 - 2 * math.log(2)), rel=1e-14)
    # deviance is nonnegative and zero exactly at x = d
    rng = np.random.default_rng(0)
    xx = rng.uniform(0, 10, 1000)
    dd = rng.poisson(5, 1000).astype(float)
    _, dv = O.objective_terms(xx, dd)
    assert np.all(dv >= -1e-12)
    _, dz = O.objective_terms(dd, dd)
    assert np.all(np.abs(dz) <= 1e-12)


def test_zero_gradient_and_objective_at_truth(c1):
    cfg, inp, d = c1
    res = O.grad(inp.obj_true, inp.probe, inp.pos, d)
    res0 = O.grad(synth.initial_object(cfg), inp.probe, inp.pos, d)
    assert abs(res["phi"]) <= 1e-10 * res0["phi"]
    assert np.linalg.norm(res["grad_obj"]) <= 1e-12 * np.linalg.norm(res0["grad_obj"])


def test_finite_difference_gradient_object_and_probe(c1):
    cfg, inp, d = c1
    psi = synth.initial_object(cfg) * 0.95 + 0.05 * inp.obj_true
    p = inp.probe * 1.1
    res = O.grad(psi, p, inp.pos, d, want_probe=True)
    for seed in range(3):
        v = _rand(psi.shape, 100 + seed)
        v *= np.linalg.norm(psi) / np.linalg.norm(v)
        h = 1e-7   # tiny intensities make the third derivative large; error is O(h^2)
        fp = O.minfunc(psi + h * v, p, inp.pos, d)[1]
        fm = O.minfunc(psi - h * v, p, inp.pos, d)[1]
        fd = (fp - fm) / (2 * h)
        an = 2 * np.vdot(res["grad_obj"], v).real
        assert abs(fd - an) <= 1e-6 * abs(an)
        q = _rand(p.shape, 200 + seed)
        q *= np.linalg.norm(p) / np.linalg.norm(q)
        fp = O.minfunc(psi, p + h * q, inp.pos, d)[1]
        fm = O.minfunc(psi, p - h * q, inp.pos, d)[1]
        fd = (fp - fm) / (2 * h)
        an = 2 * np.vdot(res["grad_probe"], q).real
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_global_phase_invariance(c1):
    cfg, inp, d = c1
    psi = 0.9 * synth.initial_object(cfg) + 0.1 * inp.obj_true
    th = 0.83
    a = O.grad(psi, inp.probe, inp.pos, d)
    b = O.grad(psi * np.exp(1j * th), inp.probe, inp.pos, d)
    assert b["phi"] == pytest.approx(a["phi"], rel=1e-12)
    assert np.linalg.norm(b["grad_obj"] - np.exp(1j * th) * a["grad_obj"]) <= 1e-12 * np.linalg.norm(a["grad_obj"])


def test_zero_data_closed_form():
    h, w, n = 40, 36, 8
    rng = np.random.default_rng(5)
    pos = np.stack([rng.integers(0, h - n + 1, 11), rng.integers(0, w - n + 1, 11)], 1)
    p = _rand((n, n), 6)
    psi = _rand((h, w), 7)
    d = np.zeros((11, n, n))
    res = O.grad(psi, p, pos, d)
    illum = O.illumination(p, pos, (h, w))
    ref_f = float(np.sum(illum * np.abs(psi) ** 2))
    assert res["f"] == pytest.approx(ref_f, rel=1e-13)
    assert res["phi"] == pytest.approx(ref_f, rel=1e-13)
    assert np.linalg.norm(res["grad_obj"] - illum * psi) <= 1e-13 * np.linalg.norm(illum * psi)


def test_residual_guard():
    g = np.array([0.0 + 0.0j, 1e-20 + 0j, 2.0 + 0j])
    d = np.array([3.0, 3.0, 2.0])
    r = O.residual(g, d)
    assert r[0] == 0.0 and r[1] == g[1]
    assert r[2] == pytest.approx(2.0 * (1 - 2.0 / 4.0))
