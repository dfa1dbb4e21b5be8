"""Adaptive IDW with even-grid kNN on MI355X (gfx950): thin Python binding.

Every call goes through the C ABI of ``include/aidw.h`` exported by the HIP
library ``libaidw.so`` in this directory.  This module only marshals
arguments: it checks that tensors are float32, contiguous and on the GPU,
allocates the output tensors with torch and passes raw device pointers and the
current HIP stream.  All computation happens in the library's kernels; if the
library cannot be loaded, every call raises (there is no fallback).

    import torch, paper_1601_05904_amd as aidw
    p = aidw.Params(k=10)
    qz = aidw.run(x, y, z, qx, qy, p)          # the whole method (Fig. 1)
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaidw.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "aidw.h")

OK, EINVAL, EDEGENERATE, ENOMEM, EDEVICE, ENONFINITE, ECAPACITY = 0, -1, -2, -3, -4, -5, -6
KMAX = 64


class AidwError(RuntimeError):
    """A non-zero aidw_status; ``code`` is the status, ``detail`` the library's message."""

    def __init__(self, code, detail):
        super().__init__("aidw status %d (%s): %s" % (code, _STATUS.get(code, "?"), detail))
        self.code = code
        self.detail = detail


_STATUS = {0: "ok", -1: "invalid argument", -2: "degenerate study area", -3: "out of device memory",
           -4: "HIP runtime error", -5: "non-finite coordinate", -6: "capacity exceeded"}


class _Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("alpha", ctypes.c_double * 5), ("r_min", ctypes.c_double),
                ("r_max", ctypes.c_double), ("area", ctypes.c_double), ("cell_width", ctypes.c_double),
                ("occupancy", ctypes.c_double)]


class _GridDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("min_x", ctypes.c_float), ("min_y", ctypes.c_float),
                ("max_x", ctypes.c_float), ("max_y", ctypes.c_float), ("area", ctypes.c_double),
                ("r_exp", ctypes.c_double), ("cell_width", ctypes.c_double), ("inv_cell_width", ctypes.c_float),
                ("ncol", ctypes.c_int32), ("nrow", ctypes.c_int32)]


class _Timing(ctypes.Structure):
    _fields_ = [("grid_ms", ctypes.c_float), ("knn_ms", ctypes.c_float), ("interp_ms", ctypes.c_float),
                ("finish_ms", ctypes.c_float), ("interp_q", ctypes.c_int32), ("interp_split", ctypes.c_int32)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("split_points", ctypes.c_int32), ("workers_per_cu", ctypes.c_int32),
                ("integer_powers", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class _Job(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("qx", ctypes.c_void_p), ("qy", ctypes.c_void_p), ("m", ctypes.c_int64), ("params", _Params),
                ("qz", ctypes.c_void_p), ("alpha_out", ctypes.c_void_p), ("r_obs_out", ctypes.c_void_p)]


class _BatchDesc(ctypes.Structure):
    _fields_ = [("njobs", ctypes.c_int32), ("total_data", ctypes.c_int64), ("total_queries", ctypes.c_int64),
                ("total_pairs", ctypes.c_double), ("total_cells", ctypes.c_int64), ("work_items", ctypes.c_int32),
                ("workers", ctypes.c_int32), ("kmax", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64),
                ("config", _BatchConfig)]


class _BatchTiming(ctypes.Structure):
    _fields_ = [("grid_ms", ctypes.c_float), ("knn_ms", ctypes.c_float), ("interp_ms", ctypes.c_float),
                ("finish_ms", ctypes.c_float)]


@dataclass
class Params:
    """aidw_params: k (Eq. 3), levels alpha_1..alpha_5 (Eq. 6), r_min / r_max (Eq. 5),
    area (Eq. 2; <= 0: bounding box), cell_width (<= 0: from occupancy), occupancy."""
    k: int = 10
    levels: tuple = (1.0, 2.0, 3.0, 4.0, 5.0)
    r_min: float = 0.0
    r_max: float = 2.0
    area: float = 0.0
    cell_width: float = 0.0
    occupancy: float = 2.0

    def _c(self):
        p = _Params()
        p.k = int(self.k)
        for i in range(5):
            p.alpha[i] = float(self.levels[i])
        p.r_min, p.r_max = float(self.r_min), float(self.r_max)
        p.area, p.cell_width, p.occupancy = float(self.area), float(self.cell_width), float(self.occupancy)
        return p


_lib = None
_VP = ctypes.c_void_p


def exported_functions():
    """Names of the functions declared in include/aidw.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**(aidw_[a-z_0-9]+)\s*\(", text, flags=re.M)))


def load(build_if_missing: bool = True):
    """Loads libaidw.so (building it once if it is absent) and declares the C ABI."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise OSError("libaidw.so not built: run __graft_entry__.build()")
        from . import build as _b
        _b.build()
    L = ctypes.CDLL(LIB_PATH)
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    P = ctypes.POINTER
    L.aidw_params_default.argtypes = [P(_Params)]
    L.aidw_params_default.restype = None
    L.aidw_build_grid.argtypes = [_VP, _VP, i64, _VP, _VP, i64, P(_Params), _VP, P(_VP)]
    L.aidw_grid_describe.argtypes = [_VP, P(_GridDesc)]
    L.aidw_grid_info.argtypes = [_VP, P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double), P(i32), P(i32)]
    L.aidw_grid_arrays.argtypes = [_VP, P(_VP), P(_VP), P(_VP), P(_VP)]
    L.aidw_grid_copy_arrays.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP]
    L.aidw_grid_destroy.argtypes = [_VP]
    L.aidw_grid_destroy.restype = None
    L.aidw_knn.argtypes = [_VP, _VP, _VP, i64, i32, _VP, _VP, _VP, _VP]
    L.aidw_knn_paper.argtypes = [_VP, _VP, _VP, i64, i32, _VP, _VP, _VP, _VP]
    L.aidw_nn_statistic.argtypes = [_VP, _VP, _VP, i64, i32, ctypes.c_double, _VP, _VP]
    L.aidw_knn_bruteforce.argtypes = [_VP, _VP, i64, _VP, _VP, i64, i32, _VP, _VP, _VP, _VP]
    L.aidw_interpolate_naive.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, i64, _VP, _VP, P(_Params), _VP, _VP, _VP,
                                         _VP]
    L.aidw_interpolate.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, i64, _VP, _VP, P(_Params), _VP, _VP, _VP, _VP]
    L.aidw_run.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, i64, P(_Params), _VP, _VP, _VP, _VP]
    L.aidw_run_noalloc.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, i64, P(_Params), _VP, _VP, _VP, _VP]
    L.aidw_set_timing.argtypes = [ctypes.c_int]
    L.aidw_last_timing.argtypes = [P(_Timing)]
    L.aidw_set_interp_config.argtypes = [i32, i32, i32]
    L.aidw_set_knn_config.argtypes = [i32]
    L.aidw_release_cached_memory.argtypes = []
    L.aidw_status_string.argtypes = [ctypes.c_int]
    L.aidw_status_string.restype = ctypes.c_char_p
    L.aidw_last_error_detail.argtypes = []
    L.aidw_last_error_detail.restype = ctypes.c_char_p
    L.aidw_version.restype = ctypes.c_char_p
    u64 = ctypes.c_uint64
    L.aidw_mlp_create.argtypes = [u64, ctypes.c_double, P(_VP)]
    L.aidw_mlp_destroy.argtypes = [_VP]
    L.aidw_mlp_destroy.restype = None
    L.aidw_mlp_set_params.argtypes = [_VP, _VP]
    L.aidw_mlp_get_params.argtypes = [_VP, _VP]
    L.aidw_mlp_save.argtypes = [_VP, ctypes.c_char_p]
    L.aidw_mlp_load.argtypes = [ctypes.c_char_p, P(_VP)]
    L.aidw_mlp_occupancy.argtypes = [_VP]
    L.aidw_mlp_occupancy.restype = ctypes.c_double
    L.aidw_features.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, _VP]
    L.aidw_mlp_forward.argtypes = [_VP, _VP, i64, _VP, _VP]
    L.aidw_mlp_gradients.argtypes = [_VP, _VP, _VP, i64, _VP, _VP]
    L.aidw_mlp_train.argtypes = [_VP, _VP, _VP, i64, i32, i32, ctypes.c_float, u64, _VP, _VP]
    L.aidw_run_learned.argtypes = [_VP, _VP, _VP, i64, _VP, _VP, i64, P(_Params), _VP, i32, ctypes.c_double, _VP, _VP,
                                   _VP, P(i64), _VP]
    L.aidw_learned_routes.argtypes = [_VP, _VP, i64, _VP, _VP, i64, P(_Params), _VP, i32, ctypes.c_double, _VP, _VP,
                                      _VP]
    L.aidw_batch_config_default.argtypes = [P(_BatchConfig)]
    L.aidw_batch_config_default.restype = None
    L.aidw_batch_create.argtypes = [P(_Job), i32, P(_BatchConfig), P(_VP)]
    L.aidw_batch_run.argtypes = [_VP, _VP]
    L.aidw_batch_job_status.argtypes = [_VP, P(i32), _VP]
    L.aidw_batch_describe.argtypes = [_VP, P(_BatchDesc)]
    L.aidw_batch_set_timing.argtypes = [_VP, i32]
    L.aidw_batch_last_timing.argtypes = [_VP, P(_BatchTiming)]
    L.aidw_batch_destroy.argtypes = [_VP]
    L.aidw_batch_destroy.restype = None
    L.aidw_run_batch.argtypes = [P(_Job), i32, P(_BatchConfig), P(i32), _VP]
    L.aidw_batch_tune.argtypes = [P(_Job), i32, P(_BatchConfig), i32, i32, P(ctypes.c_float), _VP]
    for name in ("aidw_build_grid", "aidw_nn_statistic", "aidw_grid_describe", "aidw_grid_info", "aidw_grid_arrays", "aidw_grid_copy_arrays", "aidw_knn",
                 "aidw_interpolate", "aidw_run", "aidw_knn_paper", "aidw_knn_bruteforce", "aidw_interpolate_naive",
                 "aidw_set_timing", "aidw_last_timing", "aidw_set_interp_config", "aidw_set_knn_config",
                 "aidw_run_noalloc",
                 "aidw_mlp_create", "aidw_mlp_set_params", "aidw_mlp_get_params", "aidw_mlp_save", "aidw_mlp_load",
                 "aidw_features", "aidw_mlp_forward", "aidw_mlp_gradients", "aidw_mlp_train", "aidw_run_learned",
                 "aidw_learned_routes",
                 "aidw_batch_create", "aidw_batch_run", "aidw_batch_job_status", "aidw_batch_describe",
                 "aidw_batch_set_timing", "aidw_batch_last_timing", "aidw_run_batch", "aidw_batch_tune",
                 "aidw_release_cached_memory"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st):
    if st != OK:
        raise AidwError(st, load().aidw_last_error_detail().decode())


def _dev(t, name, dtype=None):
    """Marshals a device tensor to a raw pointer (float32 / int32, 1-D, contiguous, on the GPU)."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    want = dtype or torch.float32
    if t.dtype != want:
        raise TypeError("%s must be %s (got %s)" % (name, want, t.dtype))
    if not t.is_cuda:
        raise TypeError("%s must be on the GPU" % name)
    if not t.is_contiguous():
        raise TypeError("%s must be contiguous" % name)
    return t.data_ptr()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Grid:
    """An aidw_grid handle (library-owned device memory, freed by close() / garbage collection)."""

    def __init__(self, handle, n):
        self._h = handle
        self.n = n

    @property
    def handle(self):
        if not self._h:
            raise ValueError("grid is closed")
        return self._h

    def describe(self) -> dict:
        d = _GridDesc()
        _check(load().aidw_grid_describe(self.handle, ctypes.byref(d)))
        return {f: getattr(d, f) for f, _ in _GridDesc._fields_}

    def info(self) -> dict:
        """aidw_grid_info: A, r_exp, the cell width and the grid's shape."""
        a, r, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        nc, nr = ctypes.c_int32(), ctypes.c_int32()
        _check(load().aidw_grid_info(self.handle, ctypes.byref(a), ctypes.byref(r), ctypes.byref(c), ctypes.byref(nc),
                                     ctypes.byref(nr)))
        return {"area": a.value, "r_exp": r.value, "cell_width": c.value, "ncol": nc.value, "nrow": nr.value}

    def arrays(self, stream=None):
        """Copies (cell_start, sx, sy, sidx) into new device tensors."""
        import torch
        d = self.describe()
        dev = torch.device("cuda", torch.cuda.current_device())
        cs = torch.empty(d["ncol"] * d["nrow"] + 1, dtype=torch.int32, device=dev)
        sx = torch.empty(self.n, dtype=torch.float32, device=dev)
        sy = torch.empty(self.n, dtype=torch.float32, device=dev)
        si = torch.empty(self.n, dtype=torch.int32, device=dev)
        _check(load().aidw_grid_copy_arrays(self.handle, cs.data_ptr(), sx.data_ptr(), sy.data_ptr(), si.data_ptr(),
                                            _stream(stream)))
        return cs, sx, sy, si

    def close(self):
        if self._h:
            load().aidw_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_grid(x, y, qx=None, qy=None, params: Params | None = None, stream=None) -> Grid:
    """aidw_build_grid: even grid over the data points; bounds over data and queries."""
    p = (params or Params())._c()
    m = 0 if qx is None else qx.numel()
    h = _VP()
    _check(load().aidw_build_grid(_dev(x, "x"), _dev(y, "y"), x.numel(), _dev(qx, "qx"), _dev(qy, "qy"), m,
                                  ctypes.byref(p), _stream(stream), ctypes.byref(h)))
    return Grid(h.value, x.numel())


def knn(grid: Grid, qx, qy, k: int, want_d1sq=True, want_idx=False, stream=None, paper_rule=False):
    """aidw_knn (or aidw_knn_paper, the paper's "+1 level" stop rule, when paper_rule)
    -> (r_obs [m], d1sq [m] or None, nn_idx [m, k] or None)."""
    import torch
    m = qx.numel()
    r = torch.empty(m, dtype=torch.float32, device=qx.device)
    d1 = torch.empty(m, dtype=torch.float32, device=qx.device) if want_d1sq else None
    ix = torch.empty((m, k), dtype=torch.int32, device=qx.device) if want_idx else None
    fn = load().aidw_knn_paper if paper_rule else load().aidw_knn
    _check(fn(grid.handle, _dev(qx, "qx"), _dev(qy, "qy"), m, int(k), r.data_ptr(),
              None if d1 is None else d1.data_ptr(), None if ix is None else ix.data_ptr(), _stream(stream)))
    return r, d1, ix


def nn_statistic(grid: Grid, qx, qy, k: int, clip: float = 0.0, stream=None):
    """aidw_nn_statistic: R = min(r_obs / r_exp, clip) of every query (Eq. 3, 4) -> R [m]."""
    import torch
    m = qx.numel()
    R = torch.empty(m, dtype=torch.float32, device=qx.device)
    _check(load().aidw_nn_statistic(grid.handle, _dev(qx, "qx"), _dev(qy, "qy"), m, int(k), float(clip), R.data_ptr(),
                                    _stream(stream)))
    return R


def interpolate(x, y, z, qx, qy, r_obs, d1sq, params: Params | None = None, grid: Grid | None = None,
                want_alpha=False, stream=None, naive=False):
    """aidw_interpolate (aidw_interpolate_naive, the untiled baseline, when naive)
    -> qz [m] (and alpha [m] if requested)."""
    import torch
    p = (params or Params())._c()
    m = qx.numel()
    qz = torch.empty(m, dtype=torch.float32, device=qx.device)
    al = torch.empty(m, dtype=torch.float32, device=qx.device) if want_alpha else None
    fn = load().aidw_interpolate_naive if naive else load().aidw_interpolate
    _check(fn(_dev(x, "x"), _dev(y, "y"), _dev(z, "z"), x.numel(), _dev(qx, "qx"), _dev(qy, "qy"), m,
              _dev(r_obs, "r_obs"), _dev(d1sq, "d1sq"), ctypes.byref(p), None if grid is None else grid.handle,
              qz.data_ptr(), None if al is None else al.data_ptr(), _stream(stream)))
    return (qz, al) if want_alpha else qz


def knn_bruteforce(x, y, qx, qy, k: int, want_d1sq=True, want_idx=False, stream=None):
    """aidw_knn_bruteforce (no grid, O(n m)) -> (r_obs [m], d1sq [m] or None, nn_idx [m, k] or None)."""
    import torch
    m = qx.numel()
    r = torch.empty(m, dtype=torch.float32, device=qx.device)
    d1 = torch.empty(m, dtype=torch.float32, device=qx.device) if want_d1sq else None
    ix = torch.empty((m, k), dtype=torch.int32, device=qx.device) if want_idx else None
    _check(load().aidw_knn_bruteforce(_dev(x, "x"), _dev(y, "y"), x.numel(), _dev(qx, "qx"), _dev(qy, "qy"), m,
                                      int(k), r.data_ptr(), None if d1 is None else d1.data_ptr(),
                                      None if ix is None else ix.data_ptr(), _stream(stream)))
    return r, d1, ix


def run(x, y, z, qx, qy, params: Params | None = None, want_alpha=False, want_robs=False, out=None, stream=None):
    """aidw_run: the whole method.  Returns qz, or (qz, alpha, r_obs) with the requested extras (else None)."""
    import torch
    p = (params or Params())._c()
    m = qx.numel()
    qz = out if out is not None else torch.empty(m, dtype=torch.float32, device=qx.device)
    al = torch.empty(m, dtype=torch.float32, device=qx.device) if want_alpha else None
    ro = torch.empty(m, dtype=torch.float32, device=qx.device) if want_robs else None
    _check(load().aidw_run(_dev(x, "x"), _dev(y, "y"), _dev(z, "z"), x.numel(), _dev(qx, "qx"), _dev(qy, "qy"), m,
                           ctypes.byref(p), _dev(qz, "qz"), None if al is None else al.data_ptr(),
                           None if ro is None else ro.data_ptr(), _stream(stream)))
    if want_alpha or want_robs:
        return qz, al, ro
    return qz


def run_noalloc(x, y, z, qx, qy, qz, params: Params | None = None, alpha=None, r_obs=None, stream=None):
    """aidw_run_noalloc: the whole method into the caller's outputs (qz [m]; alpha and r_obs
    [m] or None), every temporary taken from the library's fixed device array."""
    p = (params or Params())._c()
    _check(load().aidw_run_noalloc(_dev(x, "x"), _dev(y, "y"), _dev(z, "z"), x.numel(), _dev(qx, "qx"),
                                   _dev(qy, "qy"), qx.numel(), ctypes.byref(p), _dev(qz, "qz"),
                                   None if alpha is None else _dev(alpha, "alpha"),
                                   None if r_obs is None else _dev(r_obs, "r_obs"), _stream(stream)))


def set_timing(enable: bool):
    _check(load().aidw_set_timing(1 if enable else 0))


def last_timing() -> dict:
    t = _Timing()
    _check(load().aidw_last_timing(ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in _Timing._fields_}


def set_interp_config(q: int = 0, split: int = 0, integer_powers: int = -1):
    """Pair-kernel launch shape for later calls on this thread (0 = built-in choice);
    integer_powers = 0 forces the general exp2/log2 weight for every query."""
    _check(load().aidw_set_interp_config(int(q), int(split), int(integer_powers)))


def set_knn_config(lds_window: bool):
    """aidw_set_knn_config: stage each workgroup's cells in LDS in the one-lane kNN (later calls on
    this thread)."""
    _check(load().aidw_set_knn_config(1 if lds_window else 0))


def release_cached_memory():
    """aidw_release_cached_memory: frees the library's idle cached device blocks (waits for the device)."""
    _check(load().aidw_release_cached_memory())


def version() -> str:
    return load().aidw_version().decode()
