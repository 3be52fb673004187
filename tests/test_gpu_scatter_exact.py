"""Bit-exact check of the product overlap sum (the index part of Q^H, text
after Eq. gradient): integer-coded per-pattern waves go through the tile
lists and the ordered tile sum exactly as GRAD's stored waves do, and must
equal the oracle's scatter-add bit for bit (small integers: every partial
sum is exact in FP32, whatever the order).  Covered: the natural layout of
n <= 128 (with and without the conj(probe) multiply, probe = 1 so the
product is exact), the polyphase layout of 256^2 patterns, objects whose
width is not a multiple of the 64-pixel tile and whose height is not a
multiple of 16, the single-projection shape (2048^2, 128^2, 4096 positions),
the large one-GPU share (8192^2, 256^2, 16384 positions), and tiles crowded
by up to thousands of patterns (each way the tile-list sort orders a list)."""
import numpy as np
import pytest

from oracle import ptycho as O
from paper_2106_07575_amd import synth

from _gpu import dev, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    return lib()


def coded(k0, k1, n):
    """Integer-valued waves [k1 - k0, n, n]: each value depends on (k, u, v),
    so a wrong pattern, row or column index changes the sums."""
    k = np.arange(k0, k1, dtype=np.int64)[:, None, None]
    u = np.arange(n, dtype=np.int64)[None, :, None]
    v = np.arange(n, dtype=np.int64)[None, None, :]
    re = (k * 131 + u * 7 + v * 3) % 17 - 8
    im = (k * 29 + u * 5 + v * 11) % 13 - 6
    return (re + 1j * im).astype(np.complex64)


def polyphase(w):
    """Natural [k, n, n] -> the stored 256^2 layout: element (u, v) at
    (2 (u & 1) + (v & 1)) n^2 / 4 + (u / 2) (n / 2) + v / 2."""
    k, n, _ = w.shape
    return np.ascontiguousarray(w.reshape(k, n // 2, 2, n // 2, 2).transpose(0, 2, 4, 1, 3).reshape(k, n * n))


def run(P, pos, shape, n, chunk=1024, with_probe=False):
    k = len(pos)
    waves = torch.empty((k, n * n), dtype=torch.complex64, device="cuda")
    ref = np.zeros(shape, np.complex128)
    for lo in range(0, k, chunk):
        hi = min(k, lo + chunk)
        w = coded(lo, hi, n)
        waves[lo:hi] = dev(polyphase(w) if n == 256 else w.reshape(hi - lo, n * n))
        ref += O.scatter_add(w.astype(np.complex128), pos[lo:hi], shape)
    probe = dev(np.ones((n, n), np.complex64)) if (with_probe or n == 256) else None
    out = P.debug_tile_sum(waves, dev(pos), shape, probe=probe).cpu().numpy()
    assert np.abs(ref).max() < 2 ** 24
    return out, ref.astype(np.complex64)


@pytest.mark.parametrize("n,h,w,k", [(16, 40, 57, 13), (32, 90, 70, 9), (64, 130, 100, 5), (64, 70, 257, 8), (128, 300, 260, 11),
                                     (128, 417, 333, 40), (256, 400, 300, 3), (256, 611, 523, 12)])
@pytest.mark.parametrize("with_probe", [False, True])
def test_tile_sum_bit_exact_random_positions(P, n, h, w, k, with_probe):
    rng = np.random.default_rng(n + h)
    pos = np.stack([rng.integers(0, h - n + 1, k), rng.integers(0, w - n + 1, k)], 1).astype(np.int32)
    out, ref = run(P, pos, (h, w), n, with_probe=with_probe)
    assert np.array_equal(out, ref)


def test_tile_sum_bit_exact_corner_positions(P):
    # patches flush with every edge and corner of a ragged object
    n, h, w = 64, 201, 139
    pos = np.array([[0, 0], [0, w - n], [h - n, 0], [h - n, w - n], [h - n, 37], [5, w - n]], np.int32)
    out, ref = run(P, pos, (h, w), n)
    assert np.array_equal(out, ref)


def test_tile_sum_bit_exact_single_projection_shape(P):
    cfg = synth.CONFIGS["c2"]
    inp = synth.make_inputs(cfg)
    out, ref = run(P, inp.pos, (cfg.obj_h, cfg.obj_w), cfg.n)
    assert np.array_equal(out, ref)


def test_tile_sum_bit_exact_large_share_shape(P):
    cfg = synth.CONFIGS["c5"]
    inp = synth.make_inputs(cfg)
    out, ref = run(P, inp.pos, (cfg.obj_h, cfg.obj_w), cfg.n, chunk=512)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("k,hot", [(700, 60), (700, 300), (3000, 2500), (9000, 2100)])
def test_tile_sum_bit_exact_crowded_tiles(P, k, hot):
    # `hot` patterns stacked on the origin (one tile list that long) among
    # random ones on a 2048^2 object with 16^2 patterns: the tile-list sort
    # takes a list of up to 64 in one wave's lanes (hot = 60), up to 2048 in
    # LDS (hot = 300), and rebuilds a longer one by an ordered scan over all
    # patterns (hot = 2100, 2500)
    n, h, w = 16, 2048, 2048
    rng = np.random.default_rng(k + hot)
    pos = np.stack([rng.integers(0, h - n + 1, k), rng.integers(0, w - n + 1, k)], 1).astype(np.int32)
    pos[rng.choice(k, hot, replace=False)] = 0
    out, ref = run(P, pos, (h, w), n)
    assert np.array_equal(out, ref)
