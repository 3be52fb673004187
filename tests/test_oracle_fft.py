"""Pins of the oracle's unitary 2-D DFT against its definition and closed forms."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ptycho as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_fft_matches_bruteforce(n):
    x = _rand((2, n, n), 10 + n)
    ref = O.dft2_bruteforce(x)
    got = O.fft2u(x)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    refi = O.dft2_bruteforce(x, inverse=True)
    assert np.linalg.norm(O.ifft2u(x) - refi) <= 1e-13 * np.linalg.norm(refi)


def test_bruteforce_hand_cases():
    cases = json.load(open(os.path.join(GOLD, "dft_small.json")))["cases"]
    for c in cases:
        x = np.array(c["x_re"]) + 1j * np.array(c["x_im"])
        X = np.array(c["X_re"]) + 1j * np.array(c["X_im"])
        assert np.allclose(O.dft2_bruteforce(x), X, atol=1e-15)
        assert np.allclose(O.fft2u(x), X, atol=1e-15)


@pytest.mark.parametrize("n", [4, 16, 128])
def test_closed_forms(n):
    # delta at the origin -> constant 1/n
    x = np.zeros((n, n), complex)
    x[0, 0] = 1
    assert np.allclose(O.fft2u(x), 1.0 / n, atol=1e-15)
    # constant c -> c n at DC, zero elsewhere
    c = 0.3 - 1.7j
    X = O.fft2u(np.full((n, n), c))
    ref = np.zeros((n, n), complex)
    ref[0, 0] = c * n
    assert np.allclose(X, ref, atol=1e-12)
    # plane wave exp(2 pi i (a0 u + b0 v)/n) -> n at (a0, b0)
    a0, b0 = 1, n - 3
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    X = O.fft2u(np.exp(2j * math.pi * (a0 * u + b0 * v) / n))
    ref = np.zeros((n, n), complex)
    ref[a0, b0] = n
    assert np.allclose(X, ref, atol=1e-11)


@pytest.mark.parametrize("n", [16, 128, 256])
def test_parseval_and_inverse(n):
    x = _rand((3, n, n), n)
    X = O.fft2u(x)
    assert abs(np.linalg.norm(X) - np.linalg.norm(x)) <= 1e-13 * np.linalg.norm(x)
    assert np.linalg.norm(O.ifft2u(X) - x) <= 1e-13 * np.linalg.norm(x)
