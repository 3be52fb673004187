"""The C-ABI library loads and exports every entry point include/ptyg.h declares
(no compute: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptyg.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ptyg_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_method_calls():
    names = declared()
    for must in ["ptyg_forward", "ptyg_adjoint", "ptyg_grad", "ptyg_cg_solve", "ptyg_minfunc"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2106_07575_amd import ptyg
    if not os.path.exists(ptyg.lib_path()):
        pytest.skip("libptyg.so not built")
    lib = ctypes.CDLL(ptyg.lib_path())
    for name in declared():
        assert hasattr(lib, name), name
    assert set(declared()) == set(ptyg.EXPORTS)
    # host-only calls work without a GPU
    lib = ptyg.load()
    assert lib.ptyg_abi_version() == 5
    d = ptyg.Dims(2048, 2048, 128, 4096)
    sz = ptyg.workspace_size(d)
    assert sz > 4096 * 128 * 128 * 4
    bad = ptyg.Dims(64, 64, 48, 10)
    assert lib.ptyg_workspace_size(ctypes.byref(bad), None) == 0
    assert b"not in" in lib.ptyg_last_error()
    assert lib.ptyg_status_string(-2) == b"scan position outside the object"


def test_argument_errors_without_gpu():
    from paper_2106_07575_amd import ptyg
    if not os.path.exists(ptyg.lib_path()):
        pytest.skip("libptyg.so not built")
    lib = ptyg.load()
    d = ptyg.Dims(64, 64, 16, 4)
    # NULL arrays are rejected before any launch
    assert lib.ptyg_forward(ctypes.byref(d), None, None, None, None, None, 0, None) == -1
    small = ptyg.Dims(8, 8, 16, 4)
    assert lib.ptyg_forward(ctypes.byref(small), None, None, None, None, None, 0, None) == -1
    assert b"smaller than the probe" in lib.ptyg_last_error()


def test_nn_library_exports():
    """include/ptyg_nn.h: every declared entry point is exported and bound."""
    from paper_2106_07575_amd import nn, ptyg
    if not os.path.exists(ptyg.lib_path()):
        pytest.skip("libptyg.so not built")
    txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "ptyg_nn.h")).read(), flags=re.S)
    names = set(re.findall(r"\b(ptyg_[a-z0-9_]+)\s*\(", txt))
    lib = ctypes.CDLL(ptyg.lib_path())
    for name in names:
        assert hasattr(lib, name), name
    assert names == set(nn.EXPORTS)
    assert nn.weight_sizes(1, 32) == (32 * 96, 8 * 288)
    with pytest.raises(RuntimeError):
        nn.weight_sizes(0, 32)


def test_tile_list_buffers_are_length_checked():
    """The stitch's tile lists: buffer sizes come from the library, and short
    buffers are rejected before anything is launched (host-only calls)."""
    from paper_2106_07575_amd import ptyg
    if not os.path.exists(ptyg.lib_path()):
        pytest.skip("libptyg.so not built")
    lib = ctypes.CDLL(ptyg.lib_path())
    lib.ptyg_ws_tile_count.restype = ctypes.c_int64
    lib.ptyg_ws_tile_count.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.ptyg_ws_tile_list_capacity.restype = ctypes.c_int64
    lib.ptyg_ws_tile_list_capacity.argtypes = [ctypes.c_int32] * 4
    lib.ptyg_ws_tile_lists.restype = ctypes.c_int32
    lib.ptyg_ws_tile_lists.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_void_p]
    T = lib.ptyg_ws_tile_count(2048, 2048)
    assert T > 0 and lib.ptyg_ws_tile_count(2048, 4096) == 2 * T
    cap = lib.ptyg_ws_tile_list_capacity(4096, 2048, 2048, 64)
    assert cap >= T
    dummy = ctypes.create_string_buffer(16)
    p = ctypes.cast(dummy, ctypes.c_void_p)
    assert lib.ptyg_ws_tile_lists(p, 4096, 2048, 2048, 64, p, T, p, cap, None) != 0
    assert lib.ptyg_ws_tile_lists(p, 4096, 2048, 2048, 64, p, T + 1, p, cap - 1, None) != 0


def test_batched_workspace_scales_with_listed_pixels():
    """The batched search's far fields are sized by the listed-pixel capacity
    at n = 128 and 256 (host-only size queries, no GPU): at the large
    one-GPU share (8192^2, 256^2 probe, 16384 patterns, about 5.3% of the
    pixels with counts) its extra workspace stays under 8 GiB, against
    three full far fields (24 GiB) when every pixel is reserved."""
    from paper_2106_07575_amd import ptyg
    if not os.path.exists(ptyg.lib_path()):
        pytest.skip("libptyg.so not built")
    d = ptyg.Dims(8192, 8192, 256, 16384)
    px = 16384 * 256 * 256
    seq = ptyg.workspace_size(d, update_probe=True)
    full = ptyg.workspace_size(d, update_probe=True, line_search="batched")
    listed = ptyg.workspace_size(d, update_probe=True, line_search="batched", max_listed=int(0.053 * px))
    assert full - seq > 3 * px * 8
    assert listed - seq < 8 * 2 ** 30
    assert listed < full
    # below 128 the far fields are stored whole: the capacity is ignored
    s = ptyg.Dims(320, 320, 64, 49)
    assert ptyg.workspace_size(s, line_search="batched", max_listed=10) == ptyg.workspace_size(s, line_search="batched")


def test_host_limits_without_gpu():
    """Empty and oversized inputs are refused on the host: k = 0, an object
    smaller than the probe, an object of 2^31 pixels, and the batched search
    on k n^2 >= 2^31 intensities (32-bit element indices), while the same
    problem is sized for the sequential search."""
    from paper_2106_07575_amd import ptyg
    if not os.path.exists(ptyg.lib_path()):
        pytest.skip("libptyg.so not built")
    lib = ptyg.load()
    for d in (ptyg.Dims(64, 64, 16, 0), ptyg.Dims(15, 64, 16, 4), ptyg.Dims(65536, 32768, 16, 4)):
        assert lib.ptyg_workspace_size(ctypes.byref(d), None) == 0
    assert b"k=0" in lib.ptyg_last_error() or b"too large" in lib.ptyg_last_error()
    big = ptyg.Dims(8192, 8192, 256, 32768)
    assert ptyg.workspace_size(big) > 0
    opts = ptyg.CgOpts(1, 0, 1.0, 0.5, 0.0, 40, 1e-32, 0.0, 1, 0, -1)
    assert lib.ptyg_workspace_size(ctypes.byref(big), ctypes.byref(opts)) == 0
    assert b"2^31" in lib.ptyg_last_error()
    fits = ptyg.Dims(8192, 8192, 256, 32767)
    assert lib.ptyg_workspace_size(ctypes.byref(fits), ctypes.byref(opts)) > 0


def test_views_workspace_pads_ragged_pattern_counts():
    """The multi-view batch sizes any pattern count (host-only size queries):
    a count that does not fill the 8 patterns per workgroup at n = 32 gets
    the padded stacked problem plus the staged object and intensities, so it
    needs more workspace than the next full multiple, which needs none of
    that; n = 256 and a joint solve are still refused."""
    from paper_2106_07575_amd import ptyg
    if not os.path.exists(ptyg.lib_path()):
        pytest.skip("libptyg.so not built")
    lib = ptyg.load()
    opts = ptyg.CgOpts(1, 0, 1.0, 0.5, 0.0, 40, 1e-32, -1.0, 1, 0, -1)
    size = lambda k, n=32, views=3: lib.ptyg_views_workspace_size(ctypes.byref(ptyg.Dims(120, 120, n, k)), views,
                                                                  ctypes.byref(opts))
    full, ragged = size(64), size(63)
    assert full > 0 and ragged > full
    # the staged copies: 3 views + 32 zero rows of 120 complex64, 3 x 64 patterns of 32^2 float32
    assert ragged - full >= (3 * 120 + 32) * 120 * 8 + 3 * 64 * 32 * 32 * 4
    assert size(57) == ragged  # padded to the same 64 patterns per view
    assert lib.ptyg_views_workspace_size(ctypes.byref(ptyg.Dims(300, 300, 256, 4)), 3, ctypes.byref(opts)) == 0
    assert b"n <= 128" in lib.ptyg_last_error()
    joint = ptyg.CgOpts(1, 1, 1.0, 0.5, 0.0, 40, 1e-32, -1.0, 1, 0, -1)
    assert lib.ptyg_views_workspace_size(ctypes.byref(ptyg.Dims(120, 120, 32, 64)), 3, ctypes.byref(joint)) == 0
