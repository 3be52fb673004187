"""Pins of the oracle's Dai-Yuan direction, line search and CG loop
(Eqs. update, DaiYuan, linesearch, cg_ch1_1; Algorithm 1)."""
import math

import numpy as np
import pytest

from oracle import ptycho as O
from paper_2106_07575_amd import synth


def test_dai_yuan_hand_vectors():
    g_new = [np.array([1 + 1j, 2.0])]
    g_old = [np.array([1.0, 0.0])]
    eta = [np.array([1.0, 1.0])]
    # ||g_new||^2 = 2 + 4 = 6; <eta, g_new - g_old> = 1j + 2 -> Re 2 -> beta 3
    beta, rs = O.dai_yuan_beta(g_new, g_old, eta)
    assert beta == 3.0 and not rs
    # the imaginary part of <eta, dg> must not enter: eta = [i, 1] gives
    # conj(i) * i + 2 = 1 + 2 = 3 -> beta 2
    beta, rs = O.dai_yuan_beta(g_new, g_old, [np.array([1j, 1.0])])
    assert beta == 2.0 and not rs
    # non-positive denominator restarts
    beta, rs = O.dai_yuan_beta(g_new, g_old, [np.array([-1.0, -1.0])])
    assert beta == 0.0 and rs
    beta, rs = O.dai_yuan_beta(g_new, g_old, [np.array([1j, 0.0])])  # Re = 1? conj(i)*i = 1
    assert beta == 6.0 and not rs
    beta, rs = O.dai_yuan_beta(g_new, g_old, [np.array([0.0, 0.0])])
    assert beta == 0.0 and rs
    # two blocks sum
    beta, rs = O.dai_yuan_beta(g_new + [np.array([1.0])], g_old + [np.array([0.0])],
                               eta + [np.array([2.0])])
    assert beta == pytest.approx(7.0 / 4.0) and not rs


def test_dai_yuan_scale_invariance():
    rng = np.random.default_rng(3)
    a, b, e = (rng.standard_normal(50) + 1j * rng.standard_normal(50) for _ in range(3))
    e = e + (a - b)  # make the denominator positive
    b0, _ = O.dai_yuan_beta([a], [b], [e])
    b1, _ = O.dai_yuan_beta([7 * a], [7 * b], [7 * e])
    assert b1 == pytest.approx(b0, rel=1e-13)


def test_line_search_semantics():
    calls = []

    def phi(g):
        calls.append(g)
        return (g - 0.1) ** 2

    gamma, j, ok = O.line_search(phi, 0.01)
    assert calls == [0.5, 0.25, 0.125] and gamma == 0.125 and j == 3 and ok
    calls.clear()
    gamma, j, ok = O.line_search(lambda g: 1.0, 0.0, lmax=5)
    assert gamma == 0.0 and j == 5 and not ok
    # t > 0 relaxes the test: phi(0.5) = 0.16 <= 0.01 + 0.5 * 0.4
    gamma, j, ok = O.line_search(phi, 0.01, t=0.4)
    assert gamma == 0.5 and j == 1 and ok
    # gamma0 and tau are honoured: gamma in {gamma0 tau^j}
    gamma, j, ok = O.line_search(phi, 0.01, gamma0=2.0, tau=0.25)
    assert gamma == 2.0 * 0.25 ** j


@pytest.fixture(scope="module")
def c1():
    cfg = synth.CONFIGS["c1"]
    inp = synth.make_inputs(cfg)
    d = synth.make_data(cfg, np.abs(O.forward(inp.obj_true, inp.probe, inp.pos)) ** 2)
    return cfg, inp, d


def test_cg_invariants_and_convergence(c1):
    cfg, inp, d = c1
    obj0 = synth.initial_object(cfg)
    obj, _, tr = O.cg_solve(obj0, inp.probe, inp.pos, d, iters=cfg.iters)
    assert len(tr) == cfg.iters
    phis = [r["phi"] for r in tr]
    assert all(b <= a for a, b in zip(phis, phis[1:]))          # monotone (t = 0)
    assert phis[-1] < 1e-2 * phis[0]
    for r in tr:
        assert r["gamma"] in [0.5 ** j for j in range(1, 41)]
    assert tr[0]["restarted"] and tr[0]["beta"] == 0.0
    illum = O.illumination(inp.probe, inp.pos, obj.shape)
    mask = illum >= 1e-3 * illum.max()
    e0 = np.linalg.norm((O.align_phase(obj0, inp.obj_true, mask) - inp.obj_true)[mask])
    e1 = np.linalg.norm((O.align_phase(obj, inp.obj_true, mask) - inp.obj_true)[mask])
    assert e1 < 0.6 * e0


def test_cg_descent_direction_and_step_norm(c1):
    cfg, inp, d = c1
    x = synth.initial_object(cfg)
    _, _, tr = O.cg_solve(x, inp.probe, inp.pos, d, iters=4)
    # replay by hand: step norm equals gamma ||eta||, eta is a descent direction
    g_old = eta = None
    for m in range(4):
        g = O.grad(x, inp.probe, inp.pos, d)["grad_obj"]
        if m == 0:
            eta = -g
        else:
            beta, rs = O.dai_yuan_beta([g], [g_old], [eta])
            assert beta == pytest.approx(tr[m]["beta"], rel=1e-12)
            eta = -g + beta * eta
        assert np.vdot(g, eta).real < 0
        assert tr[m]["step_norm"] == pytest.approx(tr[m]["gamma"] * np.linalg.norm(eta), rel=1e-12)
        x = x + tr[m]["gamma"] * eta
        g_old = g


def test_cg_restart_after_failed_line_search(c1):
    cfg, inp, d = c1
    # with lmax = 1 and a huge gamma0 the first trial overshoots: gamma = 0
    _, _, tr = O.cg_solve(synth.initial_object(cfg), inp.probe, inp.pos, d,
                          iters=3, gamma0=1e9, lmax=1)
    assert tr[0]["gamma"] == 0.0 and tr[0]["step_norm"] == 0.0
    assert tr[1]["restarted"] and tr[1]["beta"] == 0.0


def test_joint_cg_monotone(c1):
    cfg, inp, d = c1
    p0 = np.abs(inp.probe).astype(complex)
    _, p, tr = O.cg_solve(synth.initial_object(cfg), p0, inp.pos, d, iters=6, update_probe=True)
    phis = [r["phi"] for r in tr]
    assert all(b <= a for a, b in zip(phis, phis[1:]))
    assert not np.allclose(p, p0)


# ------------------------------------------------------------------
# Joint object+probe mode and the target stop, pinned by a brute-force
# evaluation on the hand-worked 2x2 fixture (tests/golden/hand_2x2.json):
# the 2x2 unitary DFT written as its four +-1 sums, the deviance written per
# pixel, no oracle function used.  The fixture's hand-derived gradients give
# the first (steepest-descent) direction of both blocks.

def _hand():
    import json
    import os
    f = os.path.join(os.path.dirname(__file__), "golden", "hand_2x2.json")
    h = json.load(open(f))
    obj = np.array(h["obj_re"], dtype=complex)
    probe = np.array(h["probe_re"]) + 1j * np.array(h["probe_im"])
    pos = np.array(h["pos"], dtype=np.int32)
    data = np.array(h["data"], dtype=float)
    go = np.array(h["grad_obj_re"]) + 1j * np.array(h["grad_obj_im"])
    gp = np.array(h["grad_probe_re"]) + 1j * np.array(h["grad_probe_im"])
    return obj, probe, pos, data, go, gp


def _phi_bruteforce(obj, probe, pos, data):
    total = 0.0
    for k, (r, c) in enumerate(pos):
        e = [[probe[u][v] * obj[r + u][c + v] for v in range(2)] for u in range(2)]
        for a in range(2):
            for b in range(2):
                g = 0.5 * sum(e[u][v] * (-1) ** (a * u + b * v) for u in range(2) for v in range(2))
                x = abs(g) ** 2
                d = data[k][a][b]
                total += x if d == 0 else x - d - d * math.log(x / d)
    return total


def test_joint_first_iteration_bruteforce():
    obj, probe, pos, data, go, gp = _hand()
    phi0 = _phi_bruteforce(obj, probe, pos, data)
    assert phi0 == pytest.approx(4 * (10 - 5 - 5 * math.log(2)), rel=1e-14)
    # Algorithm 1 order: gamma <- tau gamma, evaluate, accept the first pass
    j, gamma = 0, 1.0
    while True:
        j += 1
        gamma *= 0.5
        phi1 = _phi_bruteforce(obj - gamma * go, probe - gamma * gp, pos, data)
        if phi1 <= phi0:
            break
    o, p, tr = O.cg_solve(obj, probe, pos, data, iters=2, update_probe=True)
    assert tr[0]["restarted"] and tr[0]["beta"] == 0.0
    assert tr[0]["gamma"] == gamma and tr[0]["halvings"] == j
    assert tr[0]["phi"] == pytest.approx(phi0, rel=1e-12)
    assert tr[1]["phi"] == pytest.approx(phi1, rel=1e-12)
    step = gamma * math.sqrt(np.sum(np.abs(go) ** 2) + np.sum(np.abs(gp) ** 2))
    assert tr[0]["step_norm"] == pytest.approx(step, rel=1e-12)
    # object-only mode from the same start takes a different step: the probe
    # block is what changes the search
    _, _, tro = O.cg_solve(obj, probe, pos, data, iters=1)
    jo, go_ = 0, 1.0
    while True:
        jo += 1
        go_ *= 0.5
        if _phi_bruteforce(obj - go_ * go, probe, pos, data) <= phi0:
            break
    assert tro[0]["gamma"] == go_ and tro[0]["halvings"] == jo


def test_target_stop_bruteforce():
    obj, probe, pos, data, go, gp = _hand()
    _, _, tr = O.cg_solve(obj, probe, pos, data, iters=3, update_probe=True)
    phi1 = tr[1]["phi"]
    assert phi1 == pytest.approx(_phi_bruteforce(obj - tr[0]["gamma"] * go, probe - tr[0]["gamma"] * gp, pos, data),
                                 rel=1e-12)
    # the stop is tested on Phi(psi_m) before the direction: at target = Phi_1
    # the solve ends after one update, just below it it takes the next one
    o1, p1, t1 = O.cg_solve(obj, probe, pos, data, iters=3, update_probe=True, target_phi=phi1 * (1 + 1e-12))
    assert len(t1) == 1
    assert np.allclose(o1, obj - tr[0]["gamma"] * go, rtol=0, atol=1e-15)
    o2, _, t2 = O.cg_solve(obj, probe, pos, data, iters=3, update_probe=True, target_phi=phi1 * (1 - 1e-9))
    assert len(t2) >= 2
    _, _, t0 = O.cg_solve(obj, probe, pos, data, iters=3, update_probe=True, target_phi=tr[0]["phi"])
    assert len(t0) == 0
