"""Pins of the oracle's Q, Q^H, G and G^H (Eq. fwd_model, text after Eq. gradient)."""
import json
import os

import numpy as np

from oracle import ptycho as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _pos(k, h, w, n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, h - n + 1, k), rng.integers(0, w - n + 1, k)], 1).astype(np.int32)


def test_gather_integer_coded_exact():
    h, w, n = 40, 57, 8              # non-square: a row/col swap fails
    obj = np.add.outer(np.arange(h), 1j * np.arange(w))
    pos = _pos(13, h, w, n, 1)
    pat = O.gather(obj, pos, n)
    for k, (r, c) in enumerate(pos):
        for u in range(n):
            for v in range(n):
                assert pat[k, u, v] == (r + u) + 1j * (c + v)


def test_scatter_integer_exact_against_pixel_loop():
    h, w, n = 30, 22, 6
    pos = _pos(17, h, w, n, 2)
    pat = np.zeros((len(pos), n, n), complex)
    for k in range(len(pos)):
        pat[k] = (k + 1) + 1j * np.arange(n * n).reshape(n, n)
    got = O.scatter_add(pat, pos, (h, w))
    ref = np.zeros((h, w), complex)
    for y in range(h):
        for x in range(w):
            for k, (r, c) in enumerate(pos):
                if r <= y < r + n and c <= x < c + n:
                    ref[y, x] += (k + 1) + 1j * ((y - r) * n + (x - c))
    assert np.array_equal(got, ref)


def test_hand_forward_fixture():
    g = json.load(open(os.path.join(GOLD, "hand_2x2.json")))
    obj = np.array(g["obj_re"], complex)
    probe = np.array(g["probe_re"]) + 1j * np.array(g["probe_im"])
    pos = np.array(g["pos"], np.int32)
    far = O.forward(obj, probe, pos)
    ref = np.array(g["far_re"]) + 1j * np.array(g["far_im"])
    assert np.allclose(far, ref, atol=1e-14)


def test_adjoint_dot_product_obj_and_probe():
    h, w, n = 48, 40, 16
    pos = _pos(21, h, w, n, 3)
    x = _rand((h, w), 4)
    p = _rand((n, n), 5)
    y = _rand((len(pos), n, n), 6)
    gx = O.forward(x, p, pos)
    ghy, gpy = O.adjoint(y, p, pos, (h, w), obj=x)
    lhs = np.vdot(gx, y)
    assert abs(lhs - np.vdot(x, ghy)) <= 1e-13 * abs(lhs)
    # p -> G(x, p) is linear in p too; its adjoint is the probe output
    q = _rand((n, n), 7)
    gq = O.forward(x, q, pos)
    lhs2 = np.vdot(gq, y)
    assert abs(lhs2 - np.vdot(q, gpy)) <= 1e-13 * abs(lhs2)


def test_normal_operator_is_illumination():
    h, w, n = 50, 50, 16
    pos = _pos(30, h, w, n, 8)
    p = _rand((n, n), 9)
    psi = _rand((h, w), 10)
    ghg, _ = O.adjoint(O.forward(psi, p, pos), p, pos, (h, w))
    illum = O.illumination(p, pos, (h, w))
    assert np.linalg.norm(ghg - illum * psi) <= 1e-13 * np.linalg.norm(ghg)


def test_uniform_object_and_parseval():
    h, w, n = 32, 32, 8
    pos = _pos(9, h, w, n, 11)
    p = _rand((n, n), 12)
    c = 0.7 - 0.2j
    g = O.forward(np.full((h, w), c), p, pos)
    assert np.allclose(g, c * O.fft2u(p)[None], atol=1e-13)
    psi = _rand((h, w), 13)
    g = O.forward(psi, p, pos)
    e = np.sum(np.abs(p[None] * O.gather(psi, pos, n)) ** 2)
    assert abs(np.sum(np.abs(g) ** 2) - e) <= 1e-12 * e
