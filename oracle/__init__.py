"""FP64 CPU oracle of the D3Q19 BGK update -- TEST INFRASTRUCTURE ONLY.

Only tests/, ``__graft_entry__.smoke()`` and bench.py's CPU-baseline leg may
import this package.  The product path (``paper_2208_05429_amd``) never does,
and this package never imports the product path.

This module is a ctypes binding of ``lbm_oracle.c`` (plain C, two arrays,
separate collide and stream loops, FP64; see its header for the model, the
paper sections each part follows and the data layout) plus numpy conveniences.
Arrays are numpy float64, C-contiguous, laid out ``f[q, x, y, z]`` and
``u[c, x, y, z]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_SRC_Q = os.path.join(_HERE, "lbm_oracle_q.c")  # D3Q15 / D3Q19 / D3Q27, chosen at run time
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

PERIODIC, WALL, MOVING_WALL = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP for timing)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unknown-pragmas",
               "-o", tmp, _SRC, _SRC_Q, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class CfgQ(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tau", ctypes.c_double), ("face", ctypes.c_int32 * 6), ("wall_u", ctypes.c_double * 3),
                ("q", ctypes.c_int32)]


class Cfg(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tau", ctypes.c_double), ("face", ctypes.c_int32 * 6), ("wall_u", ctypes.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d = P(ctypes.c_double)
        c = P(Cfg)
        L.orc_tables.argtypes = [P(ctypes.c_int32), d, P(ctypes.c_int32)]
        L.orc_set_threads.argtypes = [ctypes.c_int32]
        L.orc_threads.restype = ctypes.c_int32
        L.orc_check.argtypes = [c]
        L.orc_check.restype = ctypes.c_int32
        L.orc_equilibrium.argtypes = [ctypes.c_double, d, d]
        L.orc_collide_cell.argtypes = [c, d, d, d]
        for name, nargs in (("orc_init", 3), ("orc_collide", 3), ("orc_stream", 2), ("orc_macro", 5),
                            ("orc_sums", 2), ("orc_stream_adjoint", 2)):
            fn = getattr(L, name)
            fn.argtypes = [c] + [d] * nargs
            fn.restype = ctypes.c_int32
        L.orc_run.argtypes = [c, d, d, d, ctypes.c_int64]
        L.orc_run.restype = ctypes.c_int32
        L.orc_loss.argtypes = [c, d, d, d]
        L.orc_loss.restype = ctypes.c_double
        L.orc_loss_seed.argtypes = [c, d, d, d, d, d]
        L.orc_loss_seed.restype = ctypes.c_int32
        L.orc_collide_adjoint_cell.argtypes = [c, d, d, d, d, d]
        L.orc_adjoint_step.argtypes = [c, d, d, d, d, d]
        L.orc_adjoint_step.restype = ctypes.c_int32
        cq = P(CfgQ)
        L.orq_tables.argtypes = [ctypes.c_int32, P(ctypes.c_int32), d, P(ctypes.c_int32)]
        L.orq_tables.restype = ctypes.c_int32
        L.orq_check.argtypes = [cq]
        L.orq_check.restype = ctypes.c_int32
        for name, nargs in (("orq_init", 3), ("orq_collide", 3), ("orq_stream", 2), ("orq_macro", 5),
                            ("orq_sums", 2)):
            fn = getattr(L, name)
            fn.argtypes = [cq] + [d] * nargs
            fn.restype = ctypes.c_int32
        L.orq_run.argtypes = [cq, d, d, d, ctypes.c_int64]
        L.orq_run.restype = ctypes.c_int32
        L.orq_loss.argtypes = [cq, d, d, d]
        L.orq_loss.restype = ctypes.c_double
        L.orq_loss_seed.argtypes = [cq, d, d, d, d, d]
        L.orq_loss_seed.restype = ctypes.c_int32
        L.orq_adjoint_step.argtypes = [cq, d, d, d, d, d]
        L.orq_adjoint_step.restype = ctypes.c_int32
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _chk(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments")


def tables():
    """(c[19,3] int, w[19] float64, opp[19] int) as the oracle holds them."""
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19, np.float64)
    opp = np.zeros(19, np.int32)
    lib().orc_tables(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _p(w),
                     opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return c, w, opp


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


class Oracle:
    """One lattice configuration.  ``faces`` = (-x,+x,-y,+y,-z,+z) codes."""

    def __init__(self, shape, tau, faces=(PERIODIC,) * 6, wall_u=(0.0, 0.0, 0.0)):
        self.shape = tuple(int(s) for s in shape)
        self.N = int(np.prod(self.shape))
        self.cfg = Cfg(self.shape[0], self.shape[1], self.shape[2], float(tau),
                       (ctypes.c_int32 * 6)(*faces), (ctypes.c_double * 3)(*wall_u))
        _chk(lib().orc_check(ctypes.byref(self.cfg)), "configuration")

    def _fshape(self, k):
        return (k,) + self.shape

    def init(self, rho0=None, u0=None):
        f = np.zeros(self._fshape(19))
        r = None if rho0 is None else np.ascontiguousarray(rho0, np.float64)
        u = None if u0 is None else np.ascontiguousarray(u0, np.float64)
        _chk(lib().orc_init(ctypes.byref(self.cfg), _p(r), _p(u), _p(f)), "init")
        return f

    def run(self, f, nsteps, F=None):
        """nsteps plain collide+stream steps on a copy of f; returns the copy."""
        f = np.array(f, np.float64, order="C", copy=True)
        tmp = np.empty_like(f)
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        _chk(lib().orc_run(ctypes.byref(self.cfg), _p(Fa), _p(f), _p(tmp), int(nsteps)), "run")
        return f

    def collide(self, f, F=None):
        f = np.ascontiguousarray(f, np.float64)
        out = np.empty_like(f)
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        _chk(lib().orc_collide(ctypes.byref(self.cfg), _p(Fa), _p(f), _p(out)), "collide")
        return out

    def stream(self, fpost):
        fpost = np.ascontiguousarray(fpost, np.float64)
        out = np.empty_like(fpost)
        _chk(lib().orc_stream(ctypes.byref(self.cfg), _p(fpost), _p(out)), "stream")
        return out

    def stream_adjoint(self, lam):
        lam = np.ascontiguousarray(lam, np.float64)
        out = np.empty_like(lam)
        _chk(lib().orc_stream_adjoint(ctypes.byref(self.cfg), _p(lam), _p(out)), "stream_adjoint")
        return out

    def macro(self, f, F=None):
        f = np.ascontiguousarray(f, np.float64)
        rho = np.empty(self.shape)
        u = np.empty(self._fshape(3))
        un = np.empty(self.shape)
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        _chk(lib().orc_macro(ctypes.byref(self.cfg), _p(Fa), _p(f), _p(rho), _p(u), _p(un)), "macro")
        return rho, u, un

    def sums(self, f):
        out = np.zeros(4)
        _chk(lib().orc_sums(ctypes.byref(self.cfg), _p(np.ascontiguousarray(f, np.float64)), _p(out)), "sums")
        return out

    def loss(self, f, utarget, F=None):
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        return lib().orc_loss(ctypes.byref(self.cfg), _p(Fa), _p(np.ascontiguousarray(f, np.float64)),
                              _p(np.ascontiguousarray(utarget, np.float64)))

    def loss_seed(self, f, utarget, F=None):
        lam = np.empty(self._fshape(19))
        gF = np.zeros(self._fshape(3))
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        _chk(lib().orc_loss_seed(ctypes.byref(self.cfg), _p(Fa), _p(np.ascontiguousarray(f, np.float64)),
                                 _p(np.ascontiguousarray(utarget, np.float64)), _p(lam), _p(gF)), "loss_seed")
        return lam, gF

    def adjoint_step(self, f_t, lam_next, F=None, gradF=None):
        """Returns (lambda_t, gradF + this step's contribution)."""
        lam = np.array(lam_next, np.float64, order="C", copy=True)
        tmp = np.empty_like(lam)
        g = np.zeros(self._fshape(3)) if gradF is None else np.array(gradF, np.float64, order="C", copy=True)
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        _chk(lib().orc_adjoint_step(ctypes.byref(self.cfg), _p(Fa), _p(np.ascontiguousarray(f_t, np.float64)),
                                    _p(lam), _p(tmp), _p(g)), "adjoint_step")
        return lam, g

    # per-cell helpers -----------------------------------------------------
    def collide_cell(self, f19, F3=None):
        out = np.empty(19)
        Fa = None if F3 is None else np.ascontiguousarray(F3, np.float64)
        lib().orc_collide_cell(ctypes.byref(self.cfg), _p(np.ascontiguousarray(f19, np.float64)), _p(Fa), _p(out))
        return out

    def collide_adjoint_cell(self, f19, mu19, F3=None):
        lam = np.empty(19)
        gF = np.zeros(3)
        Fa = None if F3 is None else np.ascontiguousarray(F3, np.float64)
        lib().orc_collide_adjoint_cell(ctypes.byref(self.cfg), _p(np.ascontiguousarray(f19, np.float64)), _p(Fa),
                                       _p(np.ascontiguousarray(mu19, np.float64)), _p(lam), _p(gF))
        return lam, gF

    # whole-run gradient (reference for the GPU adjoint) ---------------------
    def loss_and_grad(self, f0, F, utarget, nsteps):
        """L(F) after nsteps from f0 and dL/dF by the discrete adjoint, storing
        every intermediate state (no checkpointing: the plain definition)."""
        states = [np.array(f0, np.float64, copy=True)]
        for _ in range(nsteps):
            states.append(self.run(states[-1], 1, F))
        L = self.loss(states[-1], utarget, F)
        lam, gF = self.loss_seed(states[-1], utarget, F)
        for t in range(nsteps - 1, -1, -1):
            lam, gF = self.adjoint_step(states[t], lam, F, gF)
        return L, gF


# --------------------------------------------------------------------------
# D3Q15 / D3Q19 / D3Q27 (lbm_oracle_q.c)
# --------------------------------------------------------------------------

def tables_q(q):
    """(c[Q,3] int, w[Q] float64, opp[Q] int) of velocity set q (15, 19 or 27)."""
    c = np.zeros((27, 3), np.int32)
    w = np.zeros(27, np.float64)
    opp = np.zeros(27, np.int32)
    n = lib().orq_tables(int(q), c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _p(w),
                         opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if n < 0:
        raise ValueError(f"no velocity set D3Q{q}")
    return c[:n], w[:n], opp[:n]


class OracleQ(Oracle):
    """Oracle over velocity set ``q`` (15, 19 or 27): init, run, collide,
    stream, macro, sums and the discrete adjoint (loss, seed, one reverse
    step; loss_and_grad as ``Oracle``)."""

    def __init__(self, shape, tau, q, faces=(PERIODIC,) * 6, wall_u=(0.0, 0.0, 0.0)):
        self.shape = tuple(int(s) for s in shape)
        self.N = int(np.prod(self.shape))
        self.Q = int(q)
        self.cfg = CfgQ(self.shape[0], self.shape[1], self.shape[2], float(tau),
                        (ctypes.c_int32 * 6)(*faces), (ctypes.c_double * 3)(*wall_u), int(q))
        _chk(lib().orq_check(ctypes.byref(self.cfg)), "configuration")

    def init(self, rho0=None, u0=None):
        f = np.zeros(self._fshape(self.Q))
        r = None if rho0 is None else np.ascontiguousarray(rho0, np.float64)
        u = None if u0 is None else np.ascontiguousarray(u0, np.float64)
        _chk(lib().orq_init(ctypes.byref(self.cfg), _p(r), _p(u), _p(f)), "init")
        return f

    def run(self, f, nsteps, F=None):
        f = np.array(f, np.float64, order="C", copy=True)
        tmp = np.empty_like(f)
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        _chk(lib().orq_run(ctypes.byref(self.cfg), _p(Fa), _p(f), _p(tmp), int(nsteps)), "run")
        return f

    def collide(self, f, F=None):
        f = np.ascontiguousarray(f, np.float64)
        out = np.empty_like(f)
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        _chk(lib().orq_collide(ctypes.byref(self.cfg), _p(Fa), _p(f), _p(out)), "collide")
        return out

    def stream(self, fpost):
        fpost = np.ascontiguousarray(fpost, np.float64)
        out = np.empty_like(fpost)
        _chk(lib().orq_stream(ctypes.byref(self.cfg), _p(fpost), _p(out)), "stream")
        return out

    def macro(self, f, F=None):
        f = np.ascontiguousarray(f, np.float64)
        rho = np.empty(self.shape)
        u = np.empty(self._fshape(3))
        un = np.empty(self.shape)
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        _chk(lib().orq_macro(ctypes.byref(self.cfg), _p(Fa), _p(f), _p(rho), _p(u), _p(un)), "macro")
        return rho, u, un

    def sums(self, f):
        out = np.zeros(4)
        _chk(lib().orq_sums(ctypes.byref(self.cfg), _p(np.ascontiguousarray(f, np.float64)), _p(out)), "sums")
        return out

    def loss(self, f, utarget, F=None):
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        return lib().orq_loss(ctypes.byref(self.cfg), _p(Fa), _p(np.ascontiguousarray(f, np.float64)),
                              _p(np.ascontiguousarray(utarget, np.float64)))

    def loss_seed(self, f, utarget, F=None):
        lam = np.empty(self._fshape(self.Q))
        gF = np.zeros(self._fshape(3))
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        _chk(lib().orq_loss_seed(ctypes.byref(self.cfg), _p(Fa), _p(np.ascontiguousarray(f, np.float64)),
                                 _p(np.ascontiguousarray(utarget, np.float64)), _p(lam), _p(gF)), "loss_seed")
        return lam, gF

    def adjoint_step(self, f_t, lam_next, F=None, gradF=None):
        """Returns (lambda_t, gradF + this step's contribution)."""
        lam = np.array(lam_next, np.float64, order="C", copy=True)
        tmp = np.empty_like(lam)
        g = np.zeros(self._fshape(3)) if gradF is None else np.array(gradF, np.float64, order="C", copy=True)
        Fa = None if F is None else np.ascontiguousarray(F, np.float64)
        _chk(lib().orq_adjoint_step(ctypes.byref(self.cfg), _p(Fa), _p(np.ascontiguousarray(f_t, np.float64)),
                                    _p(lam), _p(tmp), _p(g)), "adjoint_step")
        return lam, g

    def collide_adjoint_cell(self, *a, **k):
        raise NotImplementedError("the generic-lattice oracle's adjoint works on whole lattices")
