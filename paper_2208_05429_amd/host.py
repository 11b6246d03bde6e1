"""ctypes binding of liblbm_cpu.so (include/lbm_cpu.h): the paper's
sequential CPU algorithms, Fuse Swap (Sec. 3, Alg. 1) and the two-step
memory-aware sweep with prism traversal (Sec. 4.1, Alg. 2), as host context
for the GPU library.  Argument marshalling only; arrays are numpy float64 in
the array-of-structures layout g[x, y, z, q] holding f - w.  They are never
a fallback for the GPU path: nothing in lattice.py or adjoint.py calls them.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import capi

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_cpu.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lbm_cpu.h")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2208_05429_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        cfgp = ctypes.POINTER(capi.lbm_config)
        dp = ctypes.POINTER(ctypes.c_double)
        L.lbm_cpu_init.argtypes = [cfgp, dp, dp, dp]
        L.lbm_cpu_fuse_swap.argtypes = [cfgp, dp, ctypes.c_int64]
        L.lbm_cpu_two_step.argtypes = [cfgp, dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
        for fn in (L.lbm_cpu_init, L.lbm_cpu_fuse_swap, L.lbm_cpu_two_step):
            fn.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(st, what):
    if st != capi.LBM_OK:
        raise capi.LbmError(st, what)


def _arr(g, cfg):
    assert g.dtype == np.float64 and g.flags.c_contiguous and g.shape == (cfg.nx, cfg.ny, cfg.nz, 19)
    return g


def lbm_cpu_init(cfg, rho0=None, u0=None):
    g = np.empty((cfg.nx, cfg.ny, cfg.nz, 19))
    r = None if rho0 is None else np.ascontiguousarray(rho0, dtype=np.float64)
    u = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
    _check(lib().lbm_cpu_init(ctypes.byref(cfg), _dp(g), _dp(r), _dp(u)), "lbm_cpu_init")
    return g


def lbm_cpu_fuse_swap(cfg, g, n):
    _check(lib().lbm_cpu_fuse_swap(ctypes.byref(cfg), _dp(_arr(g, cfg)), int(n)), "lbm_cpu_fuse_swap")


def lbm_cpu_two_step(cfg, g, n, tile=0, checked=False):
    _check(lib().lbm_cpu_two_step(ctypes.byref(cfg), _dp(_arr(g, cfg)), int(n), int(tile), 1 if checked else 0),
           "lbm_cpu_two_step")


def to_soa_f(g):
    """f[q, x, y, z] (distributions, not offsets) of an array-of-structures state."""
    from .lattice import lattice_weights
    return np.moveaxis(g, 3, 0) + lattice_weights()[:, None, None, None]
