"""ctypes binding of liblbm.so with the names of include/lbm.h.

Argument marshalling only: every computation runs in the HIP library.  The
library is loaded from this package's folder on first use; if it is missing
the call raises (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lbm.h")

LBM_OK, LBM_EINVAL, LBM_EUNSUPPORTED, LBM_EDEVICE, LBM_ESTATE = 0, -1, -2, -3, -4
LBM_F64, LBM_F32, LBM_F16_OFS, LBM_BF16_OFS = 0, 1, 2, 3
LBM_TWO_ARRAY, LBM_SWAP1, LBM_SWAP2, LBM_SWAP3 = 0, 1, 2, 3
LBM_PERIODIC, LBM_WALL, LBM_MOVING_WALL = 0, 1, 2

STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_EUNSUPPORTED", -3: "LBM_EDEVICE", -4: "LBM_ESTATE"}


class lbm_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("tau", ctypes.c_double),
                ("storage", ctypes.c_int32), ("scheme", ctypes.c_int32), ("face", ctypes.c_int32 * 6),
                ("wall_u", ctypes.c_double * 3), ("use_force", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("velocities", ctypes.c_int32)]


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None
_vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2208_05429_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        cfgp = ctypes.POINTER(lbm_config)
        sz = ctypes.POINTER(ctypes.c_size_t)
        dp = ctypes.POINTER(ctypes.c_double)
        L.lbm_buffer_sizes.argtypes = [cfgp, sz, sz]
        L.lbm_init.argtypes = [cfgp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]
        L.lbm_attach.argtypes = [cfgp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]
        L.lbm_step.argtypes = [_vp, ctypes.c_int64]
        L.lbm_step_static.argtypes = [cfgp, _vp, _vp, ctypes.c_int64, _vp, ctypes.POINTER(ctypes.c_int32)]
        L.lbm_step_into.argtypes = [_vp, _vp, _vp, ctypes.c_int32]
        L.lbm_probe_copy.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.c_int32, _vp]
        L.lbm_probe_pattern.argtypes = [cfgp, _vp, ctypes.c_int32, _vp]
        L.lbm_macroscopic.argtypes = [_vp, _vp, _vp, _vp, dp]
        L.lbm_macro_adjoint.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.lbm_step_adjoint.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int32]
        L.lbm_set_stream.argtypes = [_vp, _vp]
        L.lbm_set_kernel_timing.argtypes = [_vp, ctypes.c_int32]
        L.lbm_test_force_wait_timeout.argtypes = [_vp, ctypes.c_int32]
        L.lbm_kernel_time.argtypes = [_vp, dp, ctypes.POINTER(ctypes.c_int64)]
        L.lbm_last_error.argtypes = [_vp]
        L.lbm_last_error.restype = ctypes.c_char_p
        L.lbm_destroy.argtypes = [_vp]
        L.lbm_destroy.restype = None
        for name in ("lbm_buffer_sizes", "lbm_init", "lbm_attach", "lbm_step", "lbm_step_static", "lbm_step_into",
                     "lbm_macroscopic", "lbm_macro_adjoint", "lbm_step_adjoint", "lbm_set_stream", "lbm_set_kernel_timing",
                     "lbm_kernel_time", "lbm_test_force_wait_timeout", "lbm_probe_copy", "lbm_probe_pattern"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def header_functions():
    """Names of the functions include/lbm.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lbm_status|const char\*|void)\s+(lbm_\w+)\s*\(", text, re.M)))


def make_config(shape, tau, storage=LBM_F32, scheme=LBM_SWAP2, faces=(LBM_PERIODIC,) * 6, wall_u=(0.0, 0.0, 0.0),
                use_force=False, variant=0, velocities=19):
    return lbm_config(int(shape[0]), int(shape[1]), int(shape[2]), float(tau), int(storage), int(scheme),
                      (ctypes.c_int32 * 6)(*[int(f) for f in faces]), (ctypes.c_double * 3)(*[float(v) for v in wall_u]),
                      1 if use_force else 0, int(variant), int(velocities))


def _check(status, ctx=None):
    if status != LBM_OK:
        msg = lbm_last_error(ctx)
        raise LbmError(status, msg)


def lbm_last_error(ctx=None) -> str:
    r = lib().lbm_last_error(ctx)
    return r.decode() if r else ""


def lbm_buffer_sizes(cfg: lbm_config):
    f = ctypes.c_size_t(0)
    w = ctypes.c_size_t(0)
    st = lib().lbm_buffer_sizes(ctypes.byref(cfg), ctypes.byref(f), ctypes.byref(w))
    if st != LBM_OK:
        raise LbmError(st, "lbm_buffer_sizes rejected the configuration")
    return f.value, w.value


def lbm_init(cfg, f_dev, work_dev, force_dev, rho0_dev, u0_dev, stream):
    ctx = _vp()
    st = lib().lbm_init(ctypes.byref(cfg), f_dev, work_dev, force_dev, rho0_dev, u0_dev, stream, ctypes.byref(ctx))
    _check(st, None)
    return ctx


def lbm_attach(cfg, f_dev, work_dev, force_dev, stream):
    ctx = _vp()
    st = lib().lbm_attach(ctypes.byref(cfg), f_dev, work_dev, force_dev, stream, ctypes.byref(ctx))
    _check(st, None)
    return ctx


def lbm_step(ctx, n):
    _check(lib().lbm_step(ctx, int(n)), ctx)


def lbm_step_static(cfg, f_dev, force_dev, n, stream, report_timeout=False):
    """Returns True if a hazard wait of the call gave up (only with
    report_timeout, which makes the call wait for its passes)."""
    t = ctypes.c_int32(0)
    st = lib().lbm_step_static(ctypes.byref(cfg), f_dev, force_dev, int(n), stream,
                               ctypes.byref(t) if report_timeout else None)
    _check(st, None)
    return bool(t.value)


def lbm_step_into(ctx, f_src_dev, f_dst_dev, k):
    _check(lib().lbm_step_into(ctx, f_src_dev, f_dst_dev, int(k)), ctx)


def lbm_macroscopic(ctx, rho_dev, u_dev, unorm_dev, want_sums=False):
    sums = (ctypes.c_double * 4)() if want_sums else None
    _check(lib().lbm_macroscopic(ctx, rho_dev, u_dev, unorm_dev, sums), ctx)
    return list(sums) if want_sums else None


def lbm_macro_adjoint(ctx, f_dev, grad_u_dev, lambda_dev, grad_force_dev):
    _check(lib().lbm_macro_adjoint(ctx, f_dev, grad_u_dev, lambda_dev, grad_force_dev), ctx)


def lbm_step_adjoint(ctx, f_t_dev, lambda_in_dev, lambda_out_dev, grad_force_dev, k):
    _check(lib().lbm_step_adjoint(ctx, f_t_dev, lambda_in_dev, lambda_out_dev, grad_force_dev, int(k)), ctx)


def lbm_set_stream(ctx, stream):
    _check(lib().lbm_set_stream(ctx, stream), ctx)


def lbm_set_kernel_timing(ctx, enable):
    _check(lib().lbm_set_kernel_timing(ctx, 1 if enable else 0), ctx)


def lbm_test_force_wait_timeout(ctx, enable):
    _check(lib().lbm_test_force_wait_timeout(ctx, 1 if enable else 0), ctx)


def lbm_probe_copy(src_dev, dst_dev, nbytes, blocks, stream):
    _check(lib().lbm_probe_copy(src_dev, dst_dev, int(nbytes), int(blocks), stream), None)


def lbm_probe_pattern(cfg, f_dev, steps_per_pass, stream):
    _check(lib().lbm_probe_pattern(ctypes.byref(cfg), f_dev, int(steps_per_pass), stream), None)


def lbm_kernel_time(ctx):
    """([ms of 1-, 2- and 3-step launches], [counts])"""
    ms = (ctypes.c_double * 3)()
    n = (ctypes.c_int64 * 3)()
    _check(lib().lbm_kernel_time(ctx, ms, n), ctx)
    return list(ms), list(n)


def lbm_destroy(ctx):
    lib().lbm_destroy(ctx)
