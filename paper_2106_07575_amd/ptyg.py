"""ctypes binding of libptyg.so (include/ptyg.h) over torch device tensors.

Argument marshalling only: every step of the method runs in the HIP library.
There is no CPU fallback; if the library or a GPU is missing the calls raise.
Tensors must be contiguous, on the current HIP device: complex64 for
object / probe / far field, int32 [k, 2] for scan positions (an integer-valued
float tensor is accepted and converted exactly), float32 for intensities.
Calls run on torch's current stream.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

# the in-tree build; PTYG_LIBRARY names another build of the same sources
# (the host-sanitizer variant the CPU tests load)
_LIB_PATH = os.environ.get("PTYG_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libptyg.so")
_lib = None

PTYG_OK = 0
STATUS = {0: "OK", -1: "E_INVAL", -2: "E_BOUNDS", -3: "E_HIP", -4: "E_NONFINITE", -5: "E_WORKSPACE"}


class PtygError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ptyg {STATUS.get(status, status)}: {msg}")
        self.status = status


class Dims(ctypes.Structure):
    _fields_ = [("obj_h", ctypes.c_int32), ("obj_w", ctypes.c_int32),
                ("n", ctypes.c_int32), ("k", ctypes.c_int32)]


class CgOpts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("update_probe", ctypes.c_int32),
                ("gamma0", ctypes.c_double), ("tau", ctypes.c_double), ("t", ctypes.c_double),
                ("max_halvings", ctypes.c_int32), ("eps", ctypes.c_double),
                ("target_phi", ctypes.c_double), ("line_search", ctypes.c_int32),
                ("estimator", ctypes.c_int32), ("max_listed", ctypes.c_int64)]


LINE_SEARCH = {"sequential": 0, "batched": 1}
# Poisson maximum likelihood (Eq. ML) or least squares on the amplitudes
ESTIMATOR = {"ml": 0, "ls": 1}


class IterStats(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_double), ("f_eq2", ctypes.c_double), ("gamma", ctypes.c_double),
                ("beta", ctypes.c_double), ("step_norm", ctypes.c_double),
                ("halvings", ctypes.c_int32), ("restarted", ctypes.c_int32)]


_P = ctypes.c_void_p
_SIGS = {
    "ptyg_abi_version": (ctypes.c_int32, []),
    "ptyg_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "ptyg_last_error": (ctypes.c_char_p, []),
    "ptyg_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(Dims), ctypes.POINTER(CgOpts)]),
    "ptyg_check_positions": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, ctypes.c_size_t, _P]),
    "ptyg_listed_count": (ctypes.c_int64, [ctypes.POINTER(Dims), _P, _P]),
    "ptyg_forward": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "ptyg_adjoint": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "ptyg_grad": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P, ctypes.c_float, ctypes.c_int32, _P, _P,
                                   _P, _P, ctypes.c_size_t, _P]),
    "ptyg_minfunc": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P, ctypes.c_double, _P, _P,
                                      ctypes.c_float, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P]),
    "ptyg_minfunc_noalloc": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P, ctypes.c_double, _P, _P,
                                              ctypes.c_float, ctypes.c_int32, _P, _P]),
    "ptyg_cg_solve": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P, ctypes.POINTER(CgOpts), _P,
                                       ctypes.c_size_t, ctypes.POINTER(IterStats),
                                       ctypes.POINTER(ctypes.c_int32), _P]),
    "ptyg_gd_solve": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_float, ctypes.c_int32, _P, ctypes.c_size_t,
                                       ctypes.POINTER(ctypes.c_double), _P]),
    "ptyg_views_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(Dims), ctypes.c_int32, ctypes.POINTER(CgOpts)]),
    "ptyg_cg_solve_views": (ctypes.c_int32, [ctypes.POINTER(Dims), ctypes.c_int32, _P, _P, _P, _P,
                                             ctypes.POINTER(CgOpts), _P, ctypes.c_size_t, ctypes.POINTER(IterStats),
                                             ctypes.POINTER(ctypes.c_int32), _P]),
    "ptyg_debug_gather": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P]),
    "ptyg_debug_scatter": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P]),
    "ptyg_debug_lane_swap": (ctypes.c_int32, [_P, _P, _P]),
    "ptyg_debug_grad_far": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P, ctypes.c_float, ctypes.c_int32,
                                             _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "ptyg_debug_tile_sum": (ctypes.c_int32, [ctypes.POINTER(Dims), _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "ptyg_timing_enable": (None, [ctypes.c_int32]),
    "ptyg_timing_reset": (None, []),
    "ptyg_timing_read": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.c_int32]),
}
EXPORTS = tuple(_SIGS)


def lib_path() -> str:
    return _LIB_PATH


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libptyg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2106_07575_amd.build`")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(st: int):
    if st != PTYG_OK:
        raise PtygError(st, load().ptyg_last_error().decode())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, name: str, dtype: torch.dtype) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device}); there is no CPU path")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def positions(pos: torch.Tensor) -> torch.Tensor:
    """int32 [k, 2] positions; float input must be integer-valued."""
    if pos.dtype.is_floating_point:
        if not bool(torch.all(pos == torch.round(pos))):
            raise ValueError("scan positions must be integer-valued (sub-pixel shifts are not supported)")
        pos = pos.to(torch.int32)
    if pos.dtype != torch.int32:
        pos = pos.to(torch.int32)
    if pos.dim() != 2 or pos.shape[1] != 2:
        raise ValueError("positions must have shape [k, 2]")
    return pos.contiguous()


def dims_of(obj_shape, n: int, k: int) -> Dims:
    return Dims(int(obj_shape[0]), int(obj_shape[1]), int(n), int(k))


def listed_count(data, n: int) -> int:
    """Pixels with d > 0 (or NaN) in data [k, n, n] (ptyg_listed_count)."""
    data = _dev(data, "data", torch.float32)
    d = Dims(n, n, n, data.numel() // (n * n))
    c = load().ptyg_listed_count(ctypes.byref(d), _ptr(data), _stream())
    if c < 0:
        raise PtygError(-1, load().ptyg_last_error().decode())
    return int(c)


def workspace_size(dims: Dims, update_probe: bool = False, line_search: str = "sequential",
                   max_listed: int = -1) -> int:
    o = CgOpts()
    o.update_probe = int(update_probe)
    o.line_search = LINE_SEARCH[line_search]
    o.max_listed = int(max_listed)
    sz = load().ptyg_workspace_size(ctypes.byref(dims), ctypes.byref(o))
    if sz == 0:
        raise PtygError(-1, load().ptyg_last_error().decode())
    return sz


def workspace(dims: Dims, device, update_probe: bool = False, line_search: str = "sequential",
              max_listed: int = -1) -> torch.Tensor:
    """Workspace for every call with these dims; for the batched search at
    n = 128 / 256, max_listed >= 0 sizes its far fields for that many listed
    pixels (listed_count of the data) instead of k*n*n."""
    return torch.empty(workspace_size(dims, update_probe, line_search, max_listed), dtype=torch.uint8,
                       device=device)


def _common(obj, probe, pos):
    obj = _dev(obj, "obj", torch.complex64)
    probe = _dev(probe, "probe", torch.complex64)
    pos = _dev(positions(pos), "pos", torch.int32)
    if obj.dim() != 2 or probe.dim() != 2 or probe.shape[0] != probe.shape[1]:
        raise ValueError("obj must be [H, W] and probe [n, n]")
    return obj, probe, pos, dims_of(obj.shape, probe.shape[0], pos.shape[0])


def forward(obj, probe, pos) -> torch.Tensor:
    """Far field G(obj) = F(probe * obj[pos_k]), complex64 [k, n, n]."""
    obj, probe, pos, d = _common(obj, probe, pos)
    far = torch.empty((d.k, d.n, d.n), dtype=torch.complex64, device=obj.device)
    ws = workspace(d, obj.device) if d.n == 256 else None
    _check(load().ptyg_forward(ctypes.byref(d), _ptr(obj), _ptr(probe), _ptr(pos), _ptr(far), _ptr(ws),
                               0 if ws is None else ws.numel(), _stream()))
    return far


def adjoint(far, probe, pos, obj_shape, obj=None, want_probe: bool = False):
    """(G^H far, probe adjoint or None)."""
    probe = _dev(probe, "probe", torch.complex64)
    pos = _dev(positions(pos), "pos", torch.int32)
    far = _dev(far, "far", torch.complex64)
    d = dims_of(obj_shape, probe.shape[0], pos.shape[0])
    if tuple(far.shape) != (d.k, d.n, d.n):
        raise ValueError("far must be [k, n, n]")
    out = torch.empty(tuple(obj_shape), dtype=torch.complex64, device=probe.device)
    pout = None
    if want_probe:
        if obj is None:
            raise ValueError("the probe adjoint needs obj")
        obj = _dev(obj, "obj", torch.complex64)
        pout = torch.empty_like(probe)
    ws = workspace(d, probe.device)
    _check(load().ptyg_adjoint(ctypes.byref(d), _ptr(far), _ptr(probe), _ptr(pos), _ptr(out), _ptr(obj),
                               _ptr(pout), _ptr(ws), ws.numel(), _stream()))
    return out, pout


def grad(obj, probe, pos, data, want_probe: bool = False, eps: float = 1e-32, ws=None, estimator: str = "ml"):
    """GRAD stage: returns (objective f64 [2] = (Phi, F), grad_obj, grad_probe or None)."""
    obj, probe, pos, d = _common(obj, probe, pos)
    data = _dev(data, "data", torch.float32)
    if tuple(data.shape) != (d.k, d.n, d.n):
        raise ValueError("data must be [k, n, n]")
    g = torch.empty_like(obj)
    gp = torch.empty_like(probe) if want_probe else None
    objective = torch.empty(2, dtype=torch.float64, device=obj.device)
    ws = workspace(d, obj.device) if ws is None else ws
    _check(load().ptyg_grad(ctypes.byref(d), _ptr(obj), _ptr(probe), _ptr(pos), _ptr(data), float(eps),
                            ESTIMATOR[estimator], _ptr(g), _ptr(gp), _ptr(objective), _ptr(ws), ws.numel(),
                            _stream()))
    return objective, g, gp


def minfunc(obj, probe, pos, data, dir_obj=None, dir_probe=None, gamma: float = 0.0,
            eps: float = 1e-32, ws=None, estimator: str = "ml") -> torch.Tensor:
    """Objective (Phi, F) at (obj + gamma dir_obj, probe + gamma dir_probe)."""
    obj, probe, pos, d = _common(obj, probe, pos)
    data = _dev(data, "data", torch.float32)
    if dir_obj is not None:
        dir_obj = _dev(dir_obj, "dir_obj", torch.complex64)
    if dir_probe is not None:
        dir_probe = _dev(dir_probe, "dir_probe", torch.complex64)
    objective = torch.empty(2, dtype=torch.float64, device=obj.device)
    ws = workspace(d, obj.device) if ws is None else ws
    _check(load().ptyg_minfunc(ctypes.byref(d), _ptr(obj), _ptr(dir_obj), _ptr(probe), _ptr(dir_probe),
                               float(gamma), _ptr(pos), _ptr(data), float(eps), ESTIMATOR[estimator],
                               _ptr(objective), _ptr(ws), ws.numel(), _stream()))
    return objective


def minfunc_noalloc(obj, probe, pos, data, objective, dir_obj=None, dir_probe=None, gamma: float = 0.0,
                    eps: float = 1e-32, estimator: str = "ml") -> torch.Tensor:
    """minfunc without a workspace: writes (Phi, F) into the caller's float64
    [2] device tensor `objective` and allocates nothing (n <= 128)."""
    obj, probe, pos, d = _common(obj, probe, pos)
    data = _dev(data, "data", torch.float32)
    objective = _dev(objective, "objective", torch.float64)
    if objective.numel() < 2:
        raise ValueError("objective must hold two float64 values")
    if dir_obj is not None:
        dir_obj = _dev(dir_obj, "dir_obj", torch.complex64)
    if dir_probe is not None:
        dir_probe = _dev(dir_probe, "dir_probe", torch.complex64)
    _check(load().ptyg_minfunc_noalloc(ctypes.byref(d), _ptr(obj), _ptr(dir_obj), _ptr(probe), _ptr(dir_probe),
                                       float(gamma), _ptr(pos), _ptr(data), float(eps), ESTIMATOR[estimator],
                                       _ptr(objective), _stream()))
    return objective


@dataclasses.dataclass
class CgResult:
    obj: torch.Tensor
    probe: torch.Tensor
    trace: list
    iters_done: int


def cg_solve(obj0, probe, pos, data, iters: int, update_probe: bool = False, gamma0: float = 1.0,
             tau: float = 0.5, t: float = 0.0, max_halvings: int = 40, eps: float = 1e-32,
             target_phi: float | None = None, ws=None, line_search: str = "sequential",
             estimator: str = "ml", max_listed: int | None = None) -> CgResult:
    """ML-CG (Algorithm 1).  Works on copies of obj0 / probe.  line_search:
    "sequential" (one MINFUNC pass per trial) or "batched" (trials evaluated
    from stored far fields, up to 16 per pass; the workspace must then be
    sized with the same line_search and max_listed).  max_listed: None
    sizes a new workspace from listed_count(data); with a caller workspace
    it must be the value that workspace was sized with (-1: every pixel)."""
    obj, probe_c, pos, d = _common(obj0, probe, pos)
    data = _dev(data, "data", torch.float32)
    obj = obj.clone()
    probe_c = probe_c.clone()
    if max_listed is None:
        max_listed = listed_count(data, d.n) if (line_search == "batched" and ws is None) else -1
    o = CgOpts(int(iters), int(update_probe), float(gamma0), float(tau), float(t), int(max_halvings),
               float(eps), -1.0 if target_phi is None else float(target_phi), LINE_SEARCH[line_search],
               ESTIMATOR[estimator], int(max_listed))
    ws = workspace(d, obj.device, update_probe, line_search, max_listed) if ws is None else ws
    trace = (IterStats * max(1, iters))()
    done = ctypes.c_int32(0)
    _check(load().ptyg_cg_solve(ctypes.byref(d), _ptr(obj), _ptr(probe_c), _ptr(pos), _ptr(data),
                                ctypes.byref(o), _ptr(ws), ws.numel(), trace, ctypes.byref(done), _stream()))
    rows = [{"phi": r.phi, "f": r.f_eq2, "gamma": r.gamma, "beta": r.beta, "step_norm": r.step_norm,
             "halvings": r.halvings, "restarted": bool(r.restarted)} for r in trace[:done.value]]
    return CgResult(obj, probe_c, rows, done.value)


def gd_solve(obj0, probe, pos, data, iters: int, gamma: float, update_probe: bool = False,
             eps: float = 1e-32, ws=None, estimator: str = "ml"):
    """Gradient descent (Eq. update2) with a constant step.  Works on copies;
    returns (obj, probe, [Phi at obj_m for every iteration])."""
    obj, probe_c, pos, d = _common(obj0, probe, pos)
    data = _dev(data, "data", torch.float32)
    obj = obj.clone()
    probe_c = probe_c.clone()
    ws = workspace(d, obj.device, update_probe) if ws is None else ws
    phis = (ctypes.c_double * max(1, iters))()
    _check(load().ptyg_gd_solve(ctypes.byref(d), _ptr(obj), _ptr(probe_c), _ptr(pos), _ptr(data), int(iters),
                                float(gamma), int(update_probe), float(eps), ESTIMATOR[estimator], _ptr(ws),
                                ws.numel(), phis, _stream()))
    return obj, probe_c, list(phis[:iters])


def cg_solve_views(obj0, probe, pos, data, iters: int, gamma0: float = 1.0, tau: float = 0.5, t: float = 0.0,
                   max_halvings: int = 40, eps: float = 1e-32, line_search: str = "batched",
                   estimator: str = "ml", ws=None):
    """Multi-view batch: obj0 [V, H, W], pos [V, k, 2], data [V, k, n, n],
    shared probe [n, n]; V independent ML-CG solves in one set of launches.
    Returns (obj [V, H, W], traces: V lists of row dicts, iters_done)."""
    obj = _dev(obj0, "obj", torch.complex64).clone()
    probe = _dev(probe, "probe", torch.complex64)
    pos = _dev(positions(pos.reshape(-1, 2)), "pos", torch.int32)
    data = _dev(data, "data", torch.float32)
    if obj.dim() != 3 or data.dim() != 4:
        raise ValueError("obj must be [V, H, W] and data [V, k, n, n]")
    V, H, W = obj.shape
    k = data.shape[1]
    d = dims_of((H, W), probe.shape[0], k)
    o = CgOpts(int(iters), 0, float(gamma0), float(tau), float(t), int(max_halvings), float(eps), -1.0,
               LINE_SEARCH[line_search], ESTIMATOR[estimator], -1)
    if ws is None:
        sz = load().ptyg_views_workspace_size(ctypes.byref(d), V, ctypes.byref(o))
        if sz == 0:
            raise PtygError(-1, load().ptyg_last_error().decode())
        ws = torch.empty(sz, dtype=torch.uint8, device=obj.device)
    trace = (IterStats * max(1, V * iters))()
    done = ctypes.c_int32(0)
    _check(load().ptyg_cg_solve_views(ctypes.byref(d), V, _ptr(obj), _ptr(probe), _ptr(pos), _ptr(data),
                                      ctypes.byref(o), _ptr(ws), ws.numel(), trace, ctypes.byref(done), _stream()))
    rows = [[{"phi": r.phi, "f": r.f_eq2, "gamma": r.gamma, "beta": r.beta, "step_norm": r.step_norm,
              "halvings": r.halvings, "restarted": bool(r.restarted)}
             for r in trace[v * iters: v * iters + done.value]] for v in range(V)]
    return obj, rows, done.value


def check_positions(pos, obj_shape, n: int):
    pos = _dev(positions(pos), "pos", torch.int32)
    d = dims_of(obj_shape, n, pos.shape[0])
    ws = workspace(d, pos.device)
    _check(load().ptyg_check_positions(ctypes.byref(d), _ptr(pos), _ptr(ws), ws.numel(), _stream()))


def debug_gather(obj, pos, n: int) -> torch.Tensor:
    obj = _dev(obj, "obj", torch.complex64)
    pos = _dev(positions(pos), "pos", torch.int32)
    d = dims_of(obj.shape, n, pos.shape[0])
    out = torch.empty((d.k, n, n), dtype=torch.complex64, device=obj.device)
    _check(load().ptyg_debug_gather(ctypes.byref(d), _ptr(obj), _ptr(pos), _ptr(out), _stream()))
    return out


def debug_scatter(patches, pos, obj_shape) -> torch.Tensor:
    patches = _dev(patches, "patches", torch.complex64)
    pos = _dev(positions(pos), "pos", torch.int32)
    d = dims_of(obj_shape, patches.shape[-1], pos.shape[0])
    out = torch.empty(tuple(obj_shape), dtype=torch.complex64, device=patches.device)
    _check(load().ptyg_debug_scatter(ctypes.byref(d), _ptr(patches), _ptr(pos), _ptr(out), _stream()))
    return out


def debug_grad_far(far, probe, pos, data, obj_shape, obj=None, want_probe: bool = False, eps: float = 1e-32,
                   estimator: str = "ml"):
    """GRAD from a given far field [k, n, n] (test hook): returns
    (objective f64 [2], grad_obj, grad_probe or None, residual [k, n, n])."""
    far = _dev(far, "far", torch.complex64)
    probe = _dev(probe, "probe", torch.complex64)
    pos = _dev(positions(pos), "pos", torch.int32)
    data = _dev(data, "data", torch.float32)
    d = dims_of(obj_shape, probe.shape[0], pos.shape[0])
    if tuple(far.shape) != (d.k, d.n, d.n) or tuple(data.shape) != (d.k, d.n, d.n):
        raise ValueError("far and data must be [k, n, n]")
    if want_probe:
        if obj is None:
            raise ValueError("the probe gradient needs obj")
        obj = _dev(obj, "obj", torch.complex64)
    g = torch.empty(tuple(obj_shape), dtype=torch.complex64, device=far.device)
    gp = torch.empty_like(probe) if want_probe else None
    objective = torch.empty(2, dtype=torch.float64, device=far.device)
    res = torch.empty_like(far)
    ws = workspace(d, far.device)
    _check(load().ptyg_debug_grad_far(ctypes.byref(d), _ptr(far), _ptr(probe), _ptr(pos), _ptr(data), float(eps),
                                      ESTIMATOR[estimator], _ptr(g), _ptr(obj if want_probe else None), _ptr(gp),
                                      _ptr(objective), _ptr(res), _ptr(ws), ws.numel(), _stream()))
    return objective, g, gp, res


def debug_tile_sum(waves, pos, obj_shape, probe=None) -> torch.Tensor:
    """Ordered overlap sum of per-pattern waves [k, n*n] in GRAD's stored
    layout (natural for n <= 128, polyphase for 256), times conj(probe)
    when a probe is given (test hook)."""
    waves = _dev(waves, "waves", torch.complex64)
    pos = _dev(positions(pos), "pos", torch.int32)
    k = pos.shape[0]
    n = int(round((waves.numel() // max(k, 1)) ** 0.5))
    if waves.numel() != k * n * n:
        raise ValueError("waves must hold k * n * n values")
    if probe is not None:
        probe = _dev(probe, "probe", torch.complex64)
    d = dims_of(obj_shape, n, k)
    out = torch.empty(tuple(obj_shape), dtype=torch.complex64, device=waves.device)
    ws = workspace(d, waves.device)
    _check(load().ptyg_debug_tile_sum(ctypes.byref(d), _ptr(waves), _ptr(probe), _ptr(pos), _ptr(out), _ptr(ws),
                                      ws.numel(), _stream()))
    return out


def debug_lane_swap(a, b):
    a = _dev(a, "a", torch.float32)
    b = _dev(b, "b", torch.float32)
    if a.numel() != 64 or b.numel() != 64:
        raise ValueError("lane swap operates on two float32[64] arrays")
    _check(load().ptyg_debug_lane_swap(_ptr(a), _ptr(b), _stream()))


KERNEL_KINDS = ("grad", "minfunc", "dir_forward", "tile_sum", "grad_unit")


def timing_enable(on: bool = True, kinds=None):
    """Time the kinds named in `kinds` (default: all of KERNEL_KINDS); each
    timed launch adds an event pair between kernels."""
    if not on:
        mask = 0
    elif kinds is None:
        mask = -1
    else:
        mask = 0
        for k in kinds:
            mask |= 1 << KERNEL_KINDS.index(k)
    load().ptyg_timing_enable(mask)


def timing_reset():
    load().ptyg_timing_reset()


def timing_read() -> dict:
    """{kind: (total ms, launches)} for the fused GRAD kernel, the line-search
    kernel, the direction forward transform of the batched line search, the
    ordered overlap sum of the object gradient and the whole GRAD stage
    (transform kernel + overlap sum + reductions)."""
    n = len(KERNEL_KINDS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int32 * n)()
    _check(load().ptyg_timing_read(ms, cnt, n))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS)}
