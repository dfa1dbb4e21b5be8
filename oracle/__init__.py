"""Plain FP64 CPU oracle for AIDW (arXiv 1601.05904) -- TEST INFRASTRUCTURE ONLY.

This package is the slow, obviously correct definition that the HIP library is
checked against.  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it; the library never does, and the two
share no code.

The arithmetic lives in ``aidw_oracle.c`` (compiled with
``-O2 -fno-fast-math -ffp-contract=off -fopenmp``); this module only marshals
numpy arrays through ctypes.  Each wrapper names the passage of the paper it
follows.  ``mlp.py`` holds the FP64 reference of the learned-R network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aidw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EDEGENERATE, ECAPACITY = 0, -1, -2, -6


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` (host gcc, no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64 = ctypes.c_int64
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_bounds.argtypes = [f32p, f32p, i64, f32p, f32p, i64, f64p]
        L.oracle_grid_params.restype = ctypes.c_int
        L.oracle_grid_params.argtypes = [f64p, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, f64p,
                                         ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]
        L.oracle_cell_index.argtypes = [f32p, f32p, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_int32, ctypes.c_int32, i32p]
        L.oracle_knn.argtypes = [f32p, f32p, i64, f32p, f32p, i64, ctypes.c_int32, i32p, f64p]
        L.oracle_robs.argtypes = [f64p, i64, ctypes.c_int32, f64p]
        L.oracle_knn_paper.argtypes = [f32p, f32p, i64, f32p, f32p, i64, ctypes.c_int32, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_int32, i32p, f64p]
        L.oracle_alpha.argtypes = [f64p, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, f64p,
                                   ctypes.c_void_p, ctypes.c_void_p, f64p]
        L.oracle_idw.argtypes = [f32p, f32p, f32p, i64, f32p, f32p, i64, f64p, f64p, ctypes.c_void_p]
        L.oracle_aidw.restype = ctypes.c_int
        L.oracle_aidw.argtypes = [f32p, f32p, f32p, i64, f32p, f32p, i64, ctypes.c_void_p, i64, ctypes.c_int32,
                                  f64p, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, f64p, f64p, f64p, f64p, f64p, ctypes.c_void_p, ctypes.c_void_p,
                                  f64p]
        L.oracle_features.argtypes = [f32p, f32p, i64, f32p, f32p, i64, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_int32, ctypes.c_int32, f32p]
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__("oracle status %d" % code)
        self.code = code


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_threads(t: int) -> None:
    lib().oracle_set_threads(int(t))


def bounds(x, y, qx, qy):
    """Section 4.1.1: min / max of x, y over data and queries -> (minX, minY, maxX, maxY)."""
    x, y, qx, qy = _f32(x), _f32(y), _f32(qx), _f32(qy)
    out = np.zeros(4, np.float64)
    lib().oracle_bounds(x, y, x.size, qx, qy, qx.size, out)
    return out


def grid_params(bnds, n, area=0.0, cell_width=0.0, occupancy=2.0):
    """Eq. 2 and Section 4.1.1: dict(area, r_exp, cw, inv_cw (float32), ncol, nrow)."""
    out = np.zeros(3, np.float64)
    inv = ctypes.c_float()
    nc = ctypes.c_int32()
    nr = ctypes.c_int32()
    st = lib().oracle_grid_params(_f64(bnds), int(n), float(area), float(cell_width), float(occupancy), out,
                                  ctypes.byref(inv), ctypes.byref(nc), ctypes.byref(nr))
    if st != OK:
        raise OracleError(st)
    return dict(area=out[0], r_exp=out[1], cw=out[2], inv_cw=np.float32(inv.value), ncol=nc.value, nrow=nr.value)


def cell_index(x, y, minx, miny, inv_cw, ncol, nrow):
    """Section 4.1.2: flat cell index row * nCol + col of each point (single-precision binning)."""
    x, y = _f32(x), _f32(y)
    out = np.zeros(x.size, np.int32)
    lib().oracle_cell_index(x, y, x.size, np.float32(minx), np.float32(miny), np.float32(inv_cw), int(ncol),
                            int(nrow), out)
    return out


def knn(x, y, qx, qy, k):
    """Section 2.3 brute force, (d^2, index) order -> (idx [m, k] int32, d2 [m, k] float64)."""
    x, y, qx, qy = _f32(x), _f32(y), _f32(qx), _f32(qy)
    m = qx.size
    idx = np.zeros((m, k), np.int32)
    d2 = np.zeros((m, k), np.float64)
    if m:
        lib().oracle_knn(x, y, x.size, qx, qy, m, int(k), idx, d2)
    return idx, d2


def knn_paper(x, y, qx, qy, k, minx, miny, inv_cw, ncol, nrow):
    """Section 3.2.4 as printed: level expansion to >= k points, one more level, k best in
    that block -> (idx [m, k] int32, d2 [m, k] float64).  Not exact kNN in general."""
    x, y, qx, qy = _f32(x), _f32(y), _f32(qx), _f32(qy)
    m = qx.size
    idx = np.zeros((m, k), np.int32)
    d2 = np.zeros((m, k), np.float64)
    if m:
        lib().oracle_knn_paper(x, y, x.size, qx, qy, m, int(k), np.float32(minx), np.float32(miny),
                               np.float32(inv_cw), int(ncol), int(nrow), idx, d2)
    return idx, d2


def robs(d2):
    """Eq. 3: mean of the k nearest-neighbour distances of each query."""
    d2 = _f64(d2)
    m, k = d2.shape
    out = np.zeros(m, np.float64)
    lib().oracle_robs(d2, m, k, out)
    return out


def alpha(r_obs, r_exp, r_min=0.0, r_max=2.0, levels=(1.0, 2.0, 3.0, 4.0, 5.0)):
    """Eq. 4, 5, 6 -> (R, mu, alpha)."""
    r_obs = _f64(r_obs)
    m = r_obs.size
    R = np.zeros(m)
    mu = np.zeros(m)
    a = np.zeros(m)
    lib().oracle_alpha(r_obs, m, float(r_exp), float(r_min), float(r_max), _f64(levels), _ptr(R), _ptr(mu), a)
    return R, mu, a


def idw(x, y, z, qx, qy, alpha_q, return_scale=False):
    """Eq. 1 over all data points with per-query power alpha (coincident query -> mean z of coincident points)."""
    x, y, z, qx, qy = _f32(x), _f32(y), _f32(z), _f32(qx), _f32(qy)
    m = qx.size
    a = _f64(np.broadcast_to(np.asarray(alpha_q, np.float64), (m,)))
    zq = np.zeros(m)
    s = np.zeros(m)
    lib().oracle_idw(x, y, z, x.size, qx, qy, m, a, zq, _ptr(s))
    return (zq, s) if return_scale else zq


def features(x, y, qx, qy, minx, miny, inv_cw, ncol, nrow):
    """Learned-R inputs [m, 27]: 5 x 5 cell counts around the query's cell relative to the mean
    occupancy, and the in-cell offsets (see aidw_oracle.c)."""
    x, y, qx, qy = _f32(x), _f32(y), _f32(qx), _f32(qy)
    out = np.zeros((qx.size, 27), np.float32)
    lib().oracle_features(x, y, x.size, qx, qy, qx.size, np.float32(minx), np.float32(miny), np.float32(inv_cw),
                          int(ncol), int(nrow), out)
    return out


def aidw(x, y, z, qx, qy, k=10, levels=(1.0, 2.0, 3.0, 4.0, 5.0), r_min=0.0, r_max=2.0, area=0.0,
         cell_width=0.0, occupancy=2.0, qsel=None):
    """The whole method (Fig. 1) on the selected queries; the grid bounds use ALL queries.

    Returns a dict with z, alpha, r_obs, R, s (error scale), knn_idx, knn_d2, area, r_exp, cw.
    """
    x, y, z, qx, qy = _f32(x), _f32(y), _f32(z), _f32(qx), _f32(qy)
    m = qx.size
    if qsel is None:
        sel = None
        msel = m
    else:
        sel = np.ascontiguousarray(qsel, dtype=np.int64)
        msel = sel.size
    zq, al, ro, R, s = (np.zeros(msel) for _ in range(5))
    ki = np.zeros((msel, k), np.int32)
    kd = np.zeros((msel, k), np.float64)
    sc = np.zeros(3)
    st = lib().oracle_aidw(x, y, z, x.size, qx, qy, m, _ptr(sel), msel, int(k), _f64(levels), float(r_min),
                           float(r_max), float(area), float(cell_width), float(occupancy), zq, al, ro, R, s,
                           _ptr(ki), _ptr(kd), sc)
    if st != OK:
        raise OracleError(st)
    return dict(z=zq, alpha=al, r_obs=ro, R=R, s=s, knn_idx=ki, knn_d2=kd, area=sc[0], r_exp=sc[1], cw=sc[2])
