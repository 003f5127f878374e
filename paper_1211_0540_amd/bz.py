"""Thin ctypes binding of libbz (include/bz.h), same names as the C entry points.

Only argument marshalling lives here: every step of the collision operator
runs in the library's HIP kernels.  Device buffers are torch CUDA tensors
(HIP on ROCm); streams are torch streams.  If libbz.so is missing the import
of this module fails loudly - there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libbz.so")

BZ_OK, BZ_EINVAL, BZ_EUNSUPPORTED, BZ_EDEVICE, BZ_ENOMEM, BZ_ENONFINITE, BZ_ESTATE = 0, -1, -2, -3, -4, -5, -6
BZ_W_BATCHED_F32, BZ_W_BATCHED_F64, BZ_W_PLAIN_F32, BZ_W_PLAIN_F64 = 1, 2, 3, 4
BZ_MODE_PLAIN_F64, BZ_MODE_BATCHED_F32, BZ_MODE_BATCHED_F64, BZ_MODE_PLAIN_F32 = 1, 2, 3, 4
BZ_CORE_DEFAULT, BZ_CORE_OFF = -1, -2
BZ_BATCH_FULL_SUM = 1
BZ_BATCH_FINE_SPLIT = 2
BZ_BATCH_PER_MESH = 4
SCHEDULES = {"symmetric": 0, "full": BZ_BATCH_FULL_SUM}

MODE_WEIGHTS = {BZ_MODE_PLAIN_F64: BZ_W_PLAIN_F64, BZ_MODE_BATCHED_F32: BZ_W_BATCHED_F32,
                BZ_MODE_BATCHED_F64: BZ_W_BATCHED_F64, BZ_MODE_PLAIN_F32: BZ_W_PLAIN_F32}
MODE_NAMES = {"plain_f64": BZ_MODE_PLAIN_F64, "batched_f32": BZ_MODE_BATCHED_F32,
              "batched_f64": BZ_MODE_BATCHED_F64, "plain_f32": BZ_MODE_PLAIN_F32}


class BzError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bz status {status}: {msg}")
        self.status = status


class GridInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("L", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("dv", ctypes.c_double), ("dzeta", ctypes.c_double), ("pairs", ctypes.c_longlong),
                ("core_r2", ctypes.c_int), ("core_steps", ctypes.c_longlong), ("beta", ctypes.c_double)]


class GridParams(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("L", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("core_r2", ctypes.c_int), ("beta", ctypes.c_double)]


_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_lib = None


class ClosureDesc(ctypes.Structure):
    _fields_ = [("net", ctypes.c_void_p), ("d_params", ctypes.c_void_p), ("gate", ctypes.c_double),
                ("s_in", ctypes.c_double), ("s_out", ctypes.c_double), ("judge_every", ctypes.c_int),
                ("judge_tol", ctypes.c_double), ("judge_floor", ctypes.c_double)]


class ClosureStats(ctypes.Structure):
    _fields_ = [("served", ctypes.c_uint), ("judged", ctypes.c_uint), ("failed", ctypes.c_uint),
                ("max_err", ctypes.c_float), ("unbounded", ctypes.c_uint), ("gate_cap", ctypes.c_double)]


def lib():
    """Load libbz.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is missing: build it with paper_1211_0540_amd/build.py")
    L = ctypes.CDLL(LIBPATH)
    sig = {
        "bz_api_version": (ctypes.c_int, []),
        "bz_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "bz_last_error": (ctypes.c_char_p, []),
        "bz_grid_init": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.POINTER(_vp)]),
        "bz_grid_init_ex": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           ctypes.POINTER(_vp)]),
        "bz_grid_create": (ctypes.c_int, [ctypes.POINTER(GridParams), ctypes.POINTER(_vp)]),
        "bz_grid_free": (None, [_vp]),
        "bz_weight_table_size": (_sz, [ctypes.c_int]),
        "bz_weight_table": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
        "bz_grid_query": (ctypes.c_int, [_vp, ctypes.POINTER(GridInfo)]),
        "bz_grid_coords": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "bz_weights_bytes": (_sz, [_vp, ctypes.c_int]),
        "bz_weights": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _sz, _vp]),
        "bz_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_int,
                                           ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp)]),
        "bz_batch_create_ex": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_int,
                                              ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
        "bz_batch_free": (None, [_vp]),
        "bz_batch_set_weights": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp]),
        "bz_batch_elems": (_sz, [_vp]),
        "bz_batch_cell_offset": (_sz, [_vp, ctypes.c_int]),
        "bz_workspace_bytes": (_sz, [_vp]),
        "bz_collide_batch": (ctypes.c_int, [_vp, _vp, _vp, _vp, _sz, _vp]),
        "bz_project": (ctypes.c_int, [_vp, _vp, _vp]),
        "bz_step_workspace_bytes": (_sz, [_vp]),
        "bz_step": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _vp, _sz, _vp]),
        "bz_step_check": (ctypes.c_int, [_vp, _vp, _vp]),
        "bz_transport_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, ctypes.POINTER(_vp)]),
        "bz_transport_create_ex": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                                  ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                  ctypes.POINTER(_vp)]),
        "bz_cell_moments": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
        "bz_marginal_v1": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp]),
        "bz_transport_free": (None, [_vp]),
        "bz_transport_workspace_bytes": (_sz, [_vp]),
        "bz_transport_step": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _vp, _sz, _vp]),
        "bz_strang_workspace_bytes": (_sz, [_vp, _vp]),
        "bz_strang_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _sz, _vp]),
        "bz_mlp_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
        "bz_mlp_free": (None, [_vp]),
        "bz_mlp_param_count": (_sz, [_vp]),
        "bz_mlp_param_bytes": (_sz, [_vp]),
        "bz_mlp_workspace_bytes": (_sz, [_vp, ctypes.c_int]),
        "bz_mlp_set_params": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
        "bz_mlp_get_params": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
        "bz_mlp_forward": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, _vp, _sz, _vp]),
        "bz_mlp_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp, _sz, _vp]),
        "bz_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_float, _vp]),
        "bz_closure_workspace_bytes": (_sz, [_vp, ctypes.POINTER(ClosureDesc)]),
        "bz_closure_prepare": (ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp, _vp]),
        "bz_closure_targets": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, _vp, _vp]),
        "bz_closure_collide": (ctypes.c_int, [_vp, ctypes.POINTER(ClosureDesc), _vp, _vp, _vp, _sz, _vp]),
        "bz_closure_step": (ctypes.c_int, [_vp, ctypes.POINTER(ClosureDesc), _vp, ctypes.c_double, _vp, _sz, _vp]),
        "bz_closure_strang_step": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ClosureDesc), _vp, ctypes.c_double,
                                                  ctypes.c_double, _vp, _sz, _vp]),
        "bz_closure_read_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ClosureDesc), _vp, ctypes.POINTER(ClosureStats),
                                                 _vp]),
        "bz_graph_capture_step": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
        "bz_graph_capture_strang": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _sz, _vp,
                                                   ctypes.POINTER(_vp)]),
        "bz_graph_launch": (ctypes.c_int, [_vp, _vp]),
        "bz_graph_free": (None, [_vp]),
        "bz_variant_count": (ctypes.c_int, []),
        "bz_batch_set_variant": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
        "bz_batch_get_variant": (ctypes.c_int, [_vp, ctypes.c_int]),
        "bz_batch_autotune": (ctypes.c_int, [_vp, _vp, _vp, _vp, _sz, ctypes.c_int, _vp]),
        "bz_batch_timer": (ctypes.c_int, [_vp, ctypes.c_int]),
        "bz_batch_timer_read": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
        "bz_batch_core_timer": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
        "bz_batch_one_launch": (ctypes.c_int, [_vp]),
        "bz_tuning_save": (ctypes.c_int, [ctypes.c_char_p]),
        "bz_tuning_load": (ctypes.c_int, [ctypes.c_char_p]),
        "bz_step_flags": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_uint), _vp]),
        "bz_status_str": (ctypes.c_char_p, [ctypes.c_int]),
        "bz_collide_batch_static": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
        "bz_batch_set_core_waves": (ctypes.c_int, [_vp, ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(st: int):
    if st != BZ_OK:
        raise BzError(st, lib().bz_last_error().decode())


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return _vp(int(getattr(stream, "cuda_stream", stream)))


def _dev(t, what: str):
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{what} must be a device (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


# ---------------------------------------------------------------------------
# the C entry points
# ---------------------------------------------------------------------------
def bz_api_version() -> int:
    return int(lib().bz_api_version())


def bz_grid_init(N: int, L: float, lam: float) -> int:
    h = _vp()
    _check(lib().bz_grid_init(int(N), float(L), float(lam), ctypes.byref(h)))
    return h.value


def bz_grid_init_ex(N: int, L: float, lam: float, core_r2: int = BZ_CORE_DEFAULT) -> int:
    h = _vp()
    _check(lib().bz_grid_init_ex(int(N), float(L), float(lam), int(core_r2), ctypes.byref(h)))
    return h.value


def bz_grid_create(N: int, L: float, lam: float, core_r2: int = BZ_CORE_DEFAULT, beta: float = 1.0) -> int:
    p = GridParams(int(N), float(L), float(lam), int(core_r2), float(beta))
    h = _vp()
    _check(lib().bz_grid_create(ctypes.byref(p), ctypes.byref(h)))
    return h.value


def bz_weight_table(N: int, lam: float) -> np.ndarray:
    """The universal table T_lambda(p, q) as a (3N^2/4 + 1, 3N^2 + 1) host array."""
    n = int(lib().bz_weight_table_size(int(N)))
    out = np.zeros(max(n, 1))
    _check(lib().bz_weight_table(int(N), float(lam), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(3 * N * N // 4 + 1, 3 * N * N + 1)


def bz_grid_free(g: int) -> None:
    lib().bz_grid_free(_vp(g))


def bz_grid_query(g: int) -> dict:
    info = GridInfo()
    _check(lib().bz_grid_query(_vp(g), ctypes.byref(info)))
    return {"N": info.N, "L": info.L, "lambda": info.lambda_, "dv": info.dv, "dzeta": info.dzeta,
            "pairs": info.pairs, "core_r2": info.core_r2, "core_steps": info.core_steps, "beta": info.beta}


def bz_grid_coords(g: int):
    N = bz_grid_query(g)["N"]
    v = np.zeros(N)
    z = np.zeros(N)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().bz_grid_coords(_vp(g), v.ctypes.data_as(dp), z.ctypes.data_as(dp)))
    return v, z


def bz_weights_bytes(g: int, kind: int) -> int:
    return int(lib().bz_weights_bytes(_vp(g), int(kind)))


def bz_weights(g: int, kind: int, buf, stream=None) -> None:
    _dev(buf, "weight buffer")
    nbytes = buf.numel() * buf.element_size()
    _check(lib().bz_weights(_vp(g), int(kind), _vp(_ptr(buf)), nbytes, _stream(stream)))


def bz_batch_create(grid_of_cell, grids, mode: int) -> int:
    goc = np.ascontiguousarray(grid_of_cell, dtype=np.int32)
    arr = (_vp * len(grids))(*[_vp(g) for g in grids])
    h = _vp()
    _check(lib().bz_batch_create(int(goc.size), goc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(grids),
                                 arr, int(mode), ctypes.byref(h)))
    return h.value


def bz_batch_create_ex(grid_of_cell, grids, mode: int, flags: int) -> int:
    goc = np.ascontiguousarray(grid_of_cell, dtype=np.int32)
    arr = (_vp * len(grids))(*[_vp(g) for g in grids])
    h = _vp()
    _check(lib().bz_batch_create_ex(int(goc.size), goc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    len(grids), arr, int(mode), int(flags), ctypes.byref(h)))
    return h.value


def bz_batch_free(b: int) -> None:
    lib().bz_batch_free(_vp(b))


def bz_batch_set_weights(b: int, grid_index: int, kind: int, buf) -> None:
    _dev(buf, "weight buffer")
    _check(lib().bz_batch_set_weights(_vp(b), int(grid_index), int(kind), _vp(_ptr(buf))))


def bz_batch_elems(b: int) -> int:
    return int(lib().bz_batch_elems(_vp(b)))


def bz_batch_cell_offset(b: int, cell: int) -> int:
    return int(lib().bz_batch_cell_offset(_vp(b), int(cell)))


def bz_workspace_bytes(b: int) -> int:
    return int(lib().bz_workspace_bytes(_vp(b)))


def bz_step_workspace_bytes(b: int) -> int:
    return int(lib().bz_step_workspace_bytes(_vp(b)))


def bz_collide_batch(b: int, f, qt, work, stream=None) -> None:
    for t, n in ((f, "f"), (qt, "Qt"), (work, "workspace")):
        _dev(t, n)
    _check(lib().bz_collide_batch(_vp(b), _vp(_ptr(f)), _vp(_ptr(qt)), _vp(_ptr(work)),
                                  work.numel() * work.element_size(), _stream(stream)))


def bz_project(b: int, q, stream=None) -> None:
    _dev(q, "Q")
    _check(lib().bz_project(_vp(b), _vp(_ptr(q)), _stream(stream)))


def bz_step(b: int, f, dt_over_eps: float, work, stream=None) -> None:
    _dev(f, "f")
    _dev(work, "workspace")
    _check(lib().bz_step(_vp(b), _vp(_ptr(f)), float(dt_over_eps), _vp(_ptr(work)),
                         work.numel() * work.element_size(), _stream(stream)))


def bz_step_check(b: int, work, stream=None) -> None:
    _check(lib().bz_step_check(_vp(b), _vp(_ptr(work)), _stream(stream)))


def bz_transport_create(g: int, nx: int, x_length: float, T_wall: float, far_rho: float, far_u1: float,
                        far_T: float) -> int:
    h = _vp()
    _check(lib().bz_transport_create(_vp(g), int(nx), float(x_length), float(T_wall), float(far_rho),
                                     float(far_u1), float(far_T), ctypes.byref(h)))
    return h.value


def bz_transport_create_ex(g: int, dx, T_wall: float, far_rho: float, far_u1: float, far_T: float) -> int:
    w = np.ascontiguousarray(dx, dtype=np.float64)
    h = _vp()
    _check(lib().bz_transport_create_ex(_vp(g), int(w.size), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        float(T_wall), float(far_rho), float(far_u1), float(far_T), ctypes.byref(h)))
    return h.value


def bz_cell_moments(b: int, f, mom, stream=None) -> None:
    _dev(f, "f")
    _dev(mom, "moments")
    _check(lib().bz_cell_moments(_vp(b), _vp(_ptr(f)), _vp(_ptr(mom)), _stream(stream)))


def bz_marginal_v1(b: int, f, cell: int, out, stream=None) -> None:
    _dev(f, "f")
    _dev(out, "marginal")
    _check(lib().bz_marginal_v1(_vp(b), _vp(_ptr(f)), int(cell), _vp(_ptr(out)), _stream(stream)))


def bz_transport_free(t: int) -> None:
    lib().bz_transport_free(_vp(t))


def bz_transport_workspace_bytes(t: int) -> int:
    return int(lib().bz_transport_workspace_bytes(_vp(t)))


def bz_transport_step(t: int, f, dt: float, work, stream=None) -> None:
    _dev(f, "f")
    _dev(work, "workspace")
    _check(lib().bz_transport_step(_vp(t), _vp(_ptr(f)), float(dt), _vp(_ptr(work)),
                                   work.numel() * work.element_size(), _stream(stream)))


def bz_strang_workspace_bytes(b: int, t: int) -> int:
    return int(lib().bz_strang_workspace_bytes(_vp(b), _vp(t)))


def bz_strang_step(b: int, t: int, f, dt: float, eps: float, work, stream=None) -> None:
    _dev(f, "f")
    _dev(work, "workspace")
    _check(lib().bz_strang_step(_vp(b), _vp(t), _vp(_ptr(f)), float(dt), float(eps), _vp(_ptr(work)),
                                work.numel() * work.element_size(), _stream(stream)))


def bz_mlp_create(n_in: int, n_hidden: int, n_out: int) -> int:
    h = _vp()
    _check(lib().bz_mlp_create(int(n_in), int(n_hidden), int(n_out), ctypes.byref(h)))
    return h.value


def bz_mlp_free(n: int) -> None:
    lib().bz_mlp_free(_vp(n))


def bz_mlp_param_count(n: int) -> int:
    return int(lib().bz_mlp_param_count(_vp(n)))


def bz_mlp_param_bytes(n: int) -> int:
    return int(lib().bz_mlp_param_bytes(_vp(n)))


def bz_mlp_workspace_bytes(n: int, batch: int) -> int:
    return int(lib().bz_mlp_workspace_bytes(_vp(n), int(batch)))


def bz_mlp_set_params(n: int, params, master: np.ndarray, stream=None) -> None:
    _dev(params, "parameter buffer")
    m = np.ascontiguousarray(master, dtype=np.float32)
    if m.size != bz_mlp_param_count(n):
        raise ValueError("master weight vector has the wrong length")
    _check(lib().bz_mlp_set_params(_vp(n), _vp(_ptr(params)), _vp(m.ctypes.data), _stream(stream)))


def bz_mlp_get_params(n: int, params, stream=None) -> np.ndarray:
    out = np.empty(bz_mlp_param_count(n), dtype=np.float32)
    _check(lib().bz_mlp_get_params(_vp(n), _vp(_ptr(params)), _vp(out.ctypes.data), _stream(stream)))
    return out


def bz_mlp_forward(n: int, params, x_bf16, batch: int, y, work, stream=None) -> None:
    _check(lib().bz_mlp_forward(_vp(n), _vp(_ptr(params)), _vp(_ptr(x_bf16)), int(batch), _vp(_ptr(y)),
                                _vp(_ptr(work)), work.numel() * work.element_size(), _stream(stream)))


def bz_mlp_backward(n: int, params, x_bf16, target, batch: int, grad, loss, work, stream=None) -> None:
    _check(lib().bz_mlp_backward(_vp(n), _vp(_ptr(params)), _vp(_ptr(x_bf16)), _vp(_ptr(target)), int(batch),
                                 _vp(_ptr(grad)), _vp(_ptr(loss)), _vp(_ptr(work)),
                                 work.numel() * work.element_size(), _stream(stream)))


def bz_mlp_adam(n: int, params, grad, step: int, lr: float, stream=None) -> None:
    _check(lib().bz_mlp_adam(_vp(n), _vp(_ptr(params)), _vp(_ptr(grad)), int(step), float(lr), _stream(stream)))


def bz_graph_capture_step(b: int, f, dt_over_eps: float, work, stream) -> int:
    h = _vp()
    _check(lib().bz_graph_capture_step(_vp(b), _vp(_ptr(f)), float(dt_over_eps), _vp(_ptr(work)),
                                       work.numel() * work.element_size(), _stream(stream), ctypes.byref(h)))
    return h.value


def bz_graph_capture_strang(b: int, t: int, f, dt: float, eps: float, work, stream) -> int:
    h = _vp()
    _check(lib().bz_graph_capture_strang(_vp(b), _vp(t), _vp(_ptr(f)), float(dt), float(eps), _vp(_ptr(work)),
                                         work.numel() * work.element_size(), _stream(stream), ctypes.byref(h)))
    return h.value


def bz_graph_launch(g: int, stream=None) -> None:
    _check(lib().bz_graph_launch(_vp(g), _stream(stream)))


def bz_graph_free(g: int) -> None:
    lib().bz_graph_free(_vp(g))


def closure_desc(net: int, params, gate: float, s_in: float, s_out: float, judge_every: int = 16,
                 judge_tol: float = 1e-2, judge_floor: float = 1e-3) -> ClosureDesc:
    return ClosureDesc(_vp(net), _vp(_ptr(params)), float(gate), float(s_in), float(s_out), int(judge_every),
                       float(judge_tol), float(judge_floor))


def bz_closure_workspace_bytes(b: int, desc: ClosureDesc) -> int:
    return int(lib().bz_closure_workspace_bytes(_vp(b), ctypes.byref(desc)))


def bz_closure_prepare(b: int, f, gate: float, s_in: float, state, x, stream=None) -> None:
    _check(lib().bz_closure_prepare(_vp(b), _vp(_ptr(f)), float(gate), float(s_in), _vp(_ptr(state)),
                                    _vp(_ptr(x)), _stream(stream)))


def bz_closure_targets(b: int, state, q, s_out: float, y, stream=None) -> None:
    _check(lib().bz_closure_targets(_vp(b), _vp(_ptr(state)), _vp(_ptr(q)), float(s_out), _vp(_ptr(y)),
                                    _stream(stream)))


def bz_closure_collide(b: int, desc: ClosureDesc, f, qt, work, stream=None) -> None:
    _check(lib().bz_closure_collide(_vp(b), ctypes.byref(desc), _vp(_ptr(f)), _vp(_ptr(qt)), _vp(_ptr(work)),
                                    work.numel() * work.element_size(), _stream(stream)))


def bz_closure_step(b: int, desc: ClosureDesc, f, dt_over_eps: float, work, stream=None) -> None:
    _check(lib().bz_closure_step(_vp(b), ctypes.byref(desc), _vp(_ptr(f)), float(dt_over_eps), _vp(_ptr(work)),
                                 work.numel() * work.element_size(), _stream(stream)))


def bz_closure_strang_step(b: int, t: int, desc: ClosureDesc, f, dt: float, eps: float, work, stream=None) -> None:
    _check(lib().bz_closure_strang_step(_vp(b), _vp(t), ctypes.byref(desc), _vp(_ptr(f)), float(dt), float(eps),
                                        _vp(_ptr(work)), work.numel() * work.element_size(), _stream(stream)))


def bz_closure_read_stats(b: int, desc: ClosureDesc, work, stream=None) -> dict:
    st = ClosureStats()
    _check(lib().bz_closure_read_stats(_vp(b), ctypes.byref(desc), _vp(_ptr(work)), ctypes.byref(st),
                                       _stream(stream)))
    return {"served": st.served, "judged": st.judged, "failed": st.failed, "max_err": st.max_err,
            "unbounded": st.unbounded, "gate_cap": st.gate_cap}


def mlp_pack(p: dict) -> np.ndarray:
    """Concatenate oracle-style parameters into the library's master layout."""
    return np.concatenate([np.asarray(p[k], dtype=np.float32).ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def mlp_unpack(v: np.ndarray, n_in: int, n_hidden: int, n_out: int) -> dict:
    shapes = [("W1", (n_hidden, n_in)), ("b1", (n_hidden,)), ("W2", (n_hidden, n_hidden)), ("b2", (n_hidden,)),
              ("W3", (n_out, n_hidden)), ("b3", (n_out,))]
    out, o = {}, 0
    for k, sh in shapes:
        sz = int(np.prod(sh))
        out[k] = v[o:o + sz].reshape(sh).astype(np.float64)
        o += sz
    return out


def bz_variant_count() -> int:
    return int(lib().bz_variant_count())


def bz_batch_set_variant(b: int, grid_index: int, variant: int) -> None:
    _check(lib().bz_batch_set_variant(_vp(b), int(grid_index), int(variant)))


def bz_batch_get_variant(b: int, grid_index: int) -> int:
    return int(lib().bz_batch_get_variant(_vp(b), int(grid_index)))


def bz_batch_autotune(b: int, f, qt, work, reps: int = 2, stream=None) -> None:
    _check(lib().bz_batch_autotune(_vp(b), _vp(_ptr(f)), _vp(_ptr(qt)), _vp(_ptr(work)),
                                   work.numel() * work.element_size(), int(reps), _stream(stream)))


def bz_batch_timer(b: int, enable: bool) -> None:
    _check(lib().bz_batch_timer(_vp(b), 1 if enable else 0))


def bz_batch_timer_read(b: int):
    ms = ctypes.c_double()
    n = ctypes.c_int()
    _check(lib().bz_batch_timer_read(_vp(b), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def bz_batch_set_core_waves(b: int, waves: int) -> None:
    _check(lib().bz_batch_set_core_waves(_vp(b), int(waves)))


BZ_FLAG_NONFINITE = 1
BZ_FLAG_NEGATIVE = 2


def bz_step_flags(b: int, work, stream=None) -> int:
    """BZ_FLAG_* bits of the steps since the last check (then cleared)."""
    v = ctypes.c_uint(0)
    _check(lib().bz_step_flags(_vp(b), _vp(_ptr(work)), ctypes.byref(v), _stream(stream)))
    return int(v.value)


BZ_STATIC_SCRATCH_BYTES = 256 * 1024 * 1024


def bz_collide_batch_static(b: int, f, qt, stream=None) -> None:
    """bz_collide_batch on the library's static per-GPU workspace (allocates nothing)."""
    _dev(f, "f")
    _dev(qt, "Qt")
    _check(lib().bz_collide_batch_static(_vp(b), _vp(_ptr(f)), _vp(_ptr(qt)), _stream(stream)))


def bz_tuning_save(path: str) -> None:
    _check(lib().bz_tuning_save(str(path).encode()))


def bz_tuning_load(path: str) -> None:
    _check(lib().bz_tuning_load(str(path).encode()))


def bz_batch_one_launch(b: int) -> bool:
    return bool(lib().bz_batch_one_launch(_vp(b)))


def bz_batch_core_timer(b: int):
    ms = ctypes.c_double()
    n = ctypes.c_int()
    _check(lib().bz_batch_core_timer(_vp(b), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ---------------------------------------------------------------------------
# Convenience owner of handles and device buffers (still only marshalling).
# ---------------------------------------------------------------------------
class Collision:
    """A batch of cells on one or more meshes with its weights and workspace.

    meshes: list of (N, L, lambda), (N, L, lambda, core_r2) or (N, L, lambda, core_r2, beta)
    (core_r2 and beta as in bz_grid_create; the default core and elastic collisions
    otherwise); grid_of_cell: mesh index per cell;
    mode: one of MODE_NAMES or BZ_MODE_*; schedule: "symmetric" (conjugate
    symmetry halves the batched sum, the default) or "full"; fine_split: work
    items sized for a single 64-cell group to fill the device (for batches of
    which the gated closure convolves only a few groups); per_mesh: one
    convolution launch per mesh (BZ_BATCH_PER_MESH) instead of the one launch for
    all meshes and FP64 cores.  Weight buffers may be shared between Collision
    objects through `weights_cache`.
    """

    def __init__(self, meshes, grid_of_cell, mode="batched_f32", weights_cache=None, device="cuda",
                 schedule="symmetric", fine_split=False, per_mesh=False):
        import torch
        self.mode = MODE_NAMES.get(mode, mode)
        self.kind = MODE_WEIGHTS[self.mode]
        self.meshes = [tuple(m) for m in meshes]
        self.grids = [bz_grid_create(*m) for m in self.meshes]
        self.grid_of_cell = np.asarray(grid_of_cell, dtype=np.int32)
        self.schedule = schedule
        flags = SCHEDULES[schedule] | (BZ_BATCH_FINE_SPLIT if fine_split else 0) | (BZ_BATCH_PER_MESH if per_mesh else 0)
        self.batch = bz_batch_create_ex(self.grid_of_cell, self.grids, self.mode, flags)
        cache = weights_cache if weights_cache is not None else {}
        self.weights = []
        for gi, (g, m) in enumerate(zip(self.grids, self.meshes)):
            key = (m, self.kind)
            if key not in cache:
                buf = torch.empty(bz_weights_bytes(g, self.kind), dtype=torch.uint8, device=device)
                bz_weights(g, self.kind, buf)
                cache[key] = buf
            self.weights.append(cache[key])
            bz_batch_set_weights(self.batch, gi, self.kind, cache[key])
        self.elems = bz_batch_elems(self.batch)
        self.work = torch.zeros(max(bz_step_workspace_bytes(self.batch), 256), dtype=torch.uint8, device=device)
        self.offsets = [bz_batch_cell_offset(self.batch, c) for c in range(len(self.grid_of_cell))]

    def collide(self, f, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.elems, dtype=torch.float64, device=f.device)
        bz_collide_batch(self.batch, f, out, self.work, stream)
        return out

    def project(self, q, stream=None):
        bz_project(self.batch, q, stream)
        return q

    def step(self, f, dt_over_eps, stream=None):
        bz_step(self.batch, f, dt_over_eps, self.work, stream)
        return f

    def set_variant(self, variant: int, grid_index=None):
        for gi in range(len(self.grids)) if grid_index is None else [grid_index]:
            bz_batch_set_variant(self.batch, gi, variant)

    def autotune(self, f, reps: int = 2, stream=None):
        import torch
        q = torch.empty(self.elems, dtype=torch.float64, device=f.device)
        bz_batch_autotune(self.batch, f, q, self.work, reps, stream)
        return [bz_batch_get_variant(self.batch, gi) for gi in range(len(self.grids))]

    def check(self, stream=None):
        bz_step_check(self.batch, self.work, stream)

    def strang_step(self, transport, dt, eps, f, stream=None):
        """T(dt/2) C(dt) T(dt/2) on the batch's cells (must be the transport's nx cells)."""
        need = bz_strang_workspace_bytes(self.batch, transport)
        if self.work.numel() < need:
            import torch
            self.work = torch.zeros(need, dtype=torch.uint8, device=self.work.device)
        bz_strang_step(self.batch, transport, f, dt, eps, self.work, stream)
        return f

    def pack(self, cells):
        """Concatenate per-cell (N, N, N) arrays into the batch layout (host)."""
        return np.concatenate([np.ascontiguousarray(c, dtype=np.float64).ravel() for c in cells])

    def unpack(self, flat):
        out = []
        for c, gi in enumerate(self.grid_of_cell):
            N = self.meshes[gi][0]
            o = self.offsets[c]
            out.append(flat[o:o + N ** 3].reshape(N, N, N))
        return out

    def close(self):
        if getattr(self, "batch", None):
            bz_batch_free(self.batch)
            self.batch = None
        for g in getattr(self, "grids", []):
            bz_grid_free(g)
        self.grids = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
