"""ctypes binding of the warm-start kernels (include/ptyg_nn.h) over torch
device tensors.  Marshalling only; every operation runs in libptyg.so."""
from __future__ import annotations

import ctypes

import torch

from . import ptyg

_P = ctypes.c_void_p
_I = ctypes.c_int32
_L = ctypes.c_int64
_F = ctypes.c_float
_SIGS = {
    "ptyg_nn_last_error": (ctypes.c_char_p, []),
    "ptyg_nn_weight_sizes": (_I, [_I, _I, ctypes.POINTER(_L), ctypes.POINTER(_L)]),
    "ptyg_nn_pack_weights": (_I, [_P, _I, _I, _P, _P, _P]),
    "ptyg_nn_conv3x3_fwd": (_I, [_P, _P, _P, _P, _I, _I, _I, _I, _I, _I, _I, _P]),
    "ptyg_nn_conv3x3_bwd_data": (_I, [_P, _P, _P, _I, _I, _I, _I, _I, _P]),
    "ptyg_nn_wgrad_scratch": (_L, [_I, _I, _I, _I, _I]),
    "ptyg_nn_conv3x3_bwd_weight": (_I, [_P, _P, _P, _P, _I, _I, _I, _I, _I, _P, _L, _P]),
    "ptyg_nn_relu_bwd": (_I, [_P, _P, _L, _P, _P]),
    "ptyg_nn_pool2": (_I, [_P, _P, _I, _I, _I, _I, _I, _P]),
    "ptyg_nn_up2": (_I, [_P, _P, _I, _I, _I, _I, _I, _P]),
    "ptyg_nn_input": (_I, [_P, _I, _I, _F, _P, _P]),
    "ptyg_nn_mse": (_I, [_P, _P, _L, _P, _P, _I, _P]),
    "ptyg_nn_adam": (_I, [_P, _P, _P, _P, _L, _F, _F, _F, _F, _I, _P]),
    "ptyg_ws_tile_list_capacity": (_L, [_I, _I, _I, _I]),
    "ptyg_ws_tile_count": (_L, [_I, _I]),
    "ptyg_ws_tile_lists": (_I, [_P, _I, _I, _I, _I, _P, _L, _P, _L, _P]),
    "ptyg_ws_patches": (_I, [_P, _L, _P, _P]),
    "ptyg_ws_shift_positions": (_I, [_P, _I, _I, _P, _P]),
    "ptyg_ws_phase_sync": (_I, [_P, _P, _I, _I, _I, _I, _P, _P, _P, _P, _P, _P]),
    "ptyg_ws_stitch": (_I, [_P, _P, _P, _P, _P, _I, _I, _I, _P, _P]),
    "ptyg_ws_cover_count": (_I, [_P, _I, _I, _I, _I, _P, _P, _P, _P]),
    "ptyg_ws_stitch_adjoint": (_I, [_P, _P, _P, _P, _P, _I, _I, _I, _F, _P, _P]),
}
EXPORTS = tuple(_SIGS)
_lib = None


def lib():
    global _lib
    if _lib is None:
        l = ptyg.load()
        for name, (res, args) in _SIGS.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def _ck(st):
    if st != 0:
        raise RuntimeError(f"ptyg_nn error {st}: {lib().ptyg_nn_last_error().decode()}")


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s():
    return torch.cuda.current_stream().cuda_stream


def cpad(c: int) -> int:
    return (c + 7) // 8 * 8


def weight_sizes(cin, cout):
    a, b = _L(), _L()
    _ck(lib().ptyg_nn_weight_sizes(cin, cout, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def pack_weights(w32, cin, cout, w, wt):
    _ck(lib().ptyg_nn_pack_weights(_p(w32), cin, cout, _p(w), _p(wt), _s()))


def conv_fwd(x, w, b, y, B, H, W, cin, cout, relu, out_f32=False):
    _ck(lib().ptyg_nn_conv3x3_fwd(_p(x), _p(w), _p(b), _p(y), B, H, W, cin, cout, int(relu), int(out_f32), _s()))


def conv_bwd_data(dz, wt, dx, B, H, W, cin, cout):
    _ck(lib().ptyg_nn_conv3x3_bwd_data(_p(dz), _p(wt), _p(dx), B, H, W, cin, cout, _s()))


def wgrad_scratch(B, H, W, cin, cout) -> int:
    return int(lib().ptyg_nn_wgrad_scratch(B, H, W, cin, cout))


def conv_bwd_weight(x, dz, dw, db, B, H, W, cin, cout, scratch):
    _ck(lib().ptyg_nn_conv3x3_bwd_weight(_p(x), _p(dz), _p(dw), _p(db), B, H, W, cin, cout, _p(scratch),
                                         scratch.numel() * scratch.element_size(), _s()))


def relu_bwd(dy, y, dz):
    _ck(lib().ptyg_nn_relu_bwd(_p(dy), _p(y), dy.numel(), _p(dz), _s()))


def pool2(x, y, B, H, W, c, backward=False):
    _ck(lib().ptyg_nn_pool2(_p(x), _p(y), B, H, W, c, int(backward), _s()))


def up2(x, y, B, H, W, c, backward=False):
    _ck(lib().ptyg_nn_up2(_p(x), _p(y), B, H, W, c, int(backward), _s()))


def net_input(d, x, scale):
    """d: float32 [B, n, n] patterns -> x bf16 [B, n, n, 8]."""
    _ck(lib().ptyg_nn_input(_p(d), d.shape[0], d.shape[-1], float(scale), _p(x), _s()))


def mse(out, target, dz, partials):
    _ck(lib().ptyg_nn_mse(_p(out), _p(target), target.numel() // 2, _p(dz), _p(partials), partials.numel(), _s()))


def adam(w, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    _ck(lib().ptyg_nn_adam(_p(w), _p(g), _p(m), _p(v), w.numel(), float(lr), float(b1), float(b2), float(eps),
                           int(step), _s()))


def tile_lists(wpos, H, W, q):
    """(offsets, list) int32 device tensors of the windows' tile lists."""
    K = wpos.shape[0]
    T = int(lib().ptyg_ws_tile_count(H, W))
    offsets = torch.empty(T + 1, dtype=torch.int32, device=wpos.device)
    lst = torch.empty(int(lib().ptyg_ws_tile_list_capacity(K, H, W, q)), dtype=torch.int32, device=wpos.device)
    _ck(lib().ptyg_ws_tile_lists(_p(wpos), K, H, W, q, _p(offsets), offsets.numel(), _p(lst), lst.numel(), _s()))
    return offsets, lst


def patches(out, P):
    _ck(lib().ptyg_ws_patches(_p(out), P.numel(), _p(P), _s()))


def shift_positions(pos, off, out):
    _ck(lib().ptyg_ws_shift_positions(_p(pos), pos.shape[0], int(off), _p(out), _s()))


def phase_sync(P, wpos, q, maxnb, iters, scratch):
    K = wpos.shape[0]
    z = torch.empty((K, 2), dtype=torch.float64, device=P.device)
    _ck(lib().ptyg_ws_phase_sync(_p(P), _p(wpos), K, q, maxnb, iters, _p(scratch["cnt"]), _p(scratch["nb"]),
                                 _p(scratch["c"]), _p(z), _p(scratch["ztmp"]), _s()))
    return z


def stitch(P, z, wpos, offsets, lst, H, W, q, psi0):
    _ck(lib().ptyg_ws_stitch(_p(P), _p(z), _p(wpos), _p(offsets), _p(lst), H, W, q, _p(psi0), _s()))


def cover_count(wpos, H, W, q, offsets, lst, count):
    _ck(lib().ptyg_ws_cover_count(_p(wpos), wpos.shape[0], H, W, q, _p(offsets), _p(lst), _p(count), _s()))


def stitch_adjoint(g, out, z, wpos, count, W, q, scale, dz):
    _ck(lib().ptyg_ws_stitch_adjoint(_p(g), _p(out), _p(z), _p(wpos), _p(count), wpos.shape[0], W, q,
                                     float(scale), _p(dz), _s()))
