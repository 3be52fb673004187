"""Pins of the oracle's gradient-descent solver (Eq. update2: psi_{m+1} =
psi_m - gamma grad F(psi_m), constant gamma)."""
import numpy as np

from oracle import ptycho as O
from paper_2106_07575_amd import synth


def _c1():
    cfg = synth.CONFIGS["c1"]
    inp = synth.make_inputs(cfg)
    d = synth.make_data(cfg, np.abs(O.forward(inp.obj_true, inp.probe, inp.pos)) ** 2)
    return cfg, inp, d


def test_gd_zero_data_closed_form():
    """d = 0: F = ||G psi||^2 = sum illum |psi|^2 and grad F = illum * psi
    (G^H G is the illumination), so psi_m = (1 - gamma illum)^m psi_0
    pixel by pixel and F(psi_m) = sum illum |psi_m|^2."""
    cfg, inp, _ = _c1()
    rng = np.random.default_rng(4)
    shape = inp.obj_true.shape
    psi0 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    d = np.zeros((len(inp.pos), cfg.n, cfg.n))
    illum = O.illumination(inp.probe, inp.pos, shape)
    gamma = 0.3 / illum.max()
    obj, _, tr = O.gd_solve(psi0, inp.probe, inp.pos, d, 5, gamma)
    want = (1.0 - gamma * illum) ** 5 * psi0
    assert np.abs(obj - want).max() <= 1e-12 * np.abs(want).max()
    for m, row in enumerate(tr):
        pm = (1.0 - gamma * illum) ** m * psi0
        assert abs(row["phi"] - np.sum(illum * np.abs(pm) ** 2)) <= 1e-10 * row["phi"]
        g = illum * pm
        assert abs(row["step_norm"] - gamma * np.linalg.norm(g)) <= 1e-10 * row["step_norm"]


def test_gd_zero_data_probe_step():
    """Joint mode, d = 0: grad_p F = p * sum_k |psi[s_k]|^2, one step scales
    the probe pixel by pixel."""
    cfg, inp, _ = _c1()
    rng = np.random.default_rng(5)
    shape = inp.obj_true.shape
    psi0 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    d = np.zeros((len(inp.pos), cfg.n, cfg.n))
    cover = np.sum(np.abs(O.gather(psi0, inp.pos, cfg.n)) ** 2, axis=0)
    gamma = 1e-3
    _, p1, _ = O.gd_solve(psi0, inp.probe, inp.pos, d, 1, gamma, update_probe=True)
    want = inp.probe * (1.0 - gamma * cover)
    assert np.abs(p1 - want).max() <= 1e-12 * np.abs(want).max()


def test_gd_zero_step_is_identity():
    cfg, inp, d = _c1()
    psi0 = synth.initial_object(cfg)
    obj, _, tr = O.gd_solve(psi0, inp.probe, inp.pos, d, 3, 0.0)
    assert np.array_equal(obj, psi0)
    assert tr[0]["phi"] == tr[1]["phi"] == tr[2]["phi"]


def test_gd_monotone_and_slower_than_cg():
    """A stable step (1/10 of the inverse peak illumination; 1/4 already
    overshoots on the first step, where the Poisson term's curvature exceeds
    the illumination's) decreases the objective every iteration; CG reaches
    a lower objective in the same number of iterations (the paper's
    comparison of the two solvers)."""
    cfg, inp, d = _c1()
    psi0 = synth.initial_object(cfg)
    illum = O.illumination(inp.probe, inp.pos, psi0.shape)
    gamma = 0.1 / illum.max()
    _, _, tg = O.gd_solve(psi0, inp.probe, inp.pos, d, 16, gamma)
    phis = [r["phi"] for r in tg]
    assert all(b < a for a, b in zip(phis, phis[1:]))
    _, _, tc = O.cg_solve(psi0, inp.probe, inp.pos, d, 16)
    assert tc[-1]["phi"] < tg[-1]["phi"]
