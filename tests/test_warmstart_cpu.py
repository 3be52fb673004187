"""Host-side pieces of the warm start (no GPU): the thinning of the scan
positions used to infer on a subset of patterns."""
import numpy as np

from paper_2106_07575_amd import synth
from paper_2106_07575_amd import warmstart as WS


def test_thin_positions_separation_and_order():
    cfg = synth.CONFIGS["c2"]
    pos = synth.make_inputs(cfg).pos
    idx = WS.thin_positions(pos, 40)
    assert np.all(np.diff(idx) > 0)           # scan order kept
    p = pos[idx].astype(np.int64)
    d = np.maximum(np.abs(p[:, None, 0] - p[None, :, 0]), np.abs(p[:, None, 1] - p[None, :, 1]))
    np.fill_diagonal(d, 10 ** 9)
    assert d.min() >= 40
    # every other pattern of the 64 x 64 raster (spacing 24 +- 2)
    assert len(idx) == 32 * 32


def test_thin_positions_small_separation_keeps_all():
    pos = np.array([[0, 0], [0, 10], [10, 0], [10, 10]], np.int32)
    assert list(WS.thin_positions(pos, 10)) == [0, 1, 2, 3]
    assert list(WS.thin_positions(pos, 11)) == [0]
