"""Torch-facing wrapper of the C ABI: torch owns every device buffer and the
stream; the library computes.  Argument marshalling only."""
from __future__ import annotations

import numpy as np
import torch

from . import capi

STORAGE = {"f64": capi.LBM_F64, "f32": capi.LBM_F32, "f16": capi.LBM_F16_OFS, "bf16": capi.LBM_BF16_OFS}
SCHEME = {"two_array": capi.LBM_TWO_ARRAY, "swap1": capi.LBM_SWAP1, "swap2": capi.LBM_SWAP2, "swap3": capi.LBM_SWAP3}
FACE = {"periodic": capi.LBM_PERIODIC, "wall": capi.LBM_WALL, "moving": capi.LBM_MOVING_WALL}
_STORE_DTYPE = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def real_dtype(storage: str):
    """Arithmetic type of a storage mode (forces, adjoint fields)."""
    return torch.float64 if storage == "f64" else torch.float32


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream_handle():
    return torch.cuda.current_stream().cuda_stream


class Lattice:
    """One D3Q19 lattice on the current CUDA (HIP) device.

    shape    (nx, ny, nz), x slowest
    storage  'f64' | 'f32' | 'f16' | 'bf16' (the last two store f - w)
    scheme   'two_array' | 'swap1' | 'swap2' | 'swap3' (FP32 only)
    faces    6 codes for -x,+x,-y,+y,-z,+z ('periodic' | 'wall' | 'moving')
    force    optional torch tensor (3, nx, ny, nz) of real_dtype(storage)
    rho0/u0  optional float64 tensors (nx,ny,nz) / (3,nx,ny,nz); None = 1 / 0
    velocities  19 (D3Q19), 15 or 27 (the other cubic sets)
    """

    def __init__(self, shape, tau, storage="f32", scheme="swap2", faces=("periodic",) * 6,
                 wall_u=(0.0, 0.0, 0.0), force=None, rho0=None, u0=None, variant=0, device=None, f=None,
                 velocities=19):
        self.shape = tuple(int(s) for s in shape)
        self.N = int(np.prod(self.shape))
        self.storage, self.scheme = storage, scheme
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        fcodes = [FACE[f] if isinstance(f, str) else int(f) for f in faces]
        self.Q = int(velocities)
        self.cfg = capi.make_config(self.shape, tau, STORAGE[storage], SCHEME[scheme], fcodes, wall_u,
                                    force is not None, variant, self.Q)
        fb, wb = capi.lbm_buffer_sizes(self.cfg)
        dt = _STORE_DTYPE[storage]
        if f is None:
            self.f = torch.empty((self.Q,) + self.shape, dtype=dt, device=self.device)
        else:
            assert f.dtype == dt and f.is_contiguous() and tuple(f.shape) == (self.Q,) + self.shape
            self.f = f
        assert self.f.numel() * self.f.element_size() == fb
        self.work = torch.empty(max(wb, 256), dtype=torch.uint8, device=self.device)
        self.force = None
        if force is not None:
            self.force = force.to(device=self.device, dtype=real_dtype(storage)).contiguous()
        if f is None:
            r = None if rho0 is None else torch.as_tensor(rho0, dtype=torch.float64, device=self.device).contiguous()
            u = None if u0 is None else torch.as_tensor(u0, dtype=torch.float64, device=self.device).contiguous()
            self.ctx = capi.lbm_init(self.cfg, _ptr(self.f), _ptr(self.work), _ptr(self.force), _ptr(r), _ptr(u),
                                     _stream_handle())
            torch.cuda.current_stream().synchronize()  # rho0/u0 may be freed after this call
        else:
            self.ctx = capi.lbm_attach(self.cfg, _ptr(self.f), _ptr(self.work), _ptr(self.force), _stream_handle())

    def close(self):
        if getattr(self, "ctx", None):
            capi.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int):
        capi.lbm_set_stream(self.ctx, _stream_handle())
        capi.lbm_step(self.ctx, n)

    def step_into(self, src, dst, k: int):
        """k in {1, 2} steps from state tensor src into dst (out of place; self.f untouched)."""
        capi.lbm_set_stream(self.ctx, _stream_handle())
        capi.lbm_step_into(self.ctx, _ptr(src), _ptr(dst), k)

    def macroscopic(self, sums=False, want=("rho", "u", "unorm")):
        capi.lbm_set_stream(self.ctx, _stream_handle())
        rho = torch.empty(self.shape, dtype=torch.float64, device=self.device) if "rho" in want else None
        u = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device) if "u" in want else None
        un = torch.empty(self.shape, dtype=torch.float64, device=self.device) if "unorm" in want else None
        s = capi.lbm_macroscopic(self.ctx, _ptr(rho), _ptr(u), _ptr(un), sums)
        return rho, u, un, (np.array(s) if sums else None)

    def set_kernel_timing(self, enable=True):
        capi.lbm_set_kernel_timing(self.ctx, enable)

    def kernel_time(self):
        """Summed ms and counts of the update-kernel launches since timing was enabled."""
        return capi.lbm_kernel_time(self.ctx)

    def sums(self):
        return self.macroscopic(sums=True, want=())[3]

    def distributions(self):
        """f = g + w as float64 (host numpy), layout [q, x, y, z]."""
        g = self.f.to(torch.float64).cpu().numpy()
        return g + lattice_weights(self.Q)[:, None, None, None]


def lattice_weights(q=19):
    """Weights of velocity set D3Q{q} in the library's direction order."""
    c2 = (lattice_velocities(q) ** 2).sum(axis=1)
    by_speed = {15: (2 / 9, 1 / 9, 0.0, 1 / 72), 19: (1 / 3, 1 / 18, 1 / 36, 0.0),
                27: (8 / 27, 2 / 27, 1 / 54, 1 / 216)}[q]
    return np.array([by_speed[s] for s in c2])


def lattice_velocities(q=19):
    """The direction order of include/lbm.h (interface, not arithmetic)."""
    half = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (-1, -1, 0), (-1, 1, 0), (-1, 0, -1), (-1, 0, 1), (0, -1, -1),
            (0, -1, 1)]
    corners = [(-1, -1, -1), (-1, -1, 1), (-1, 1, -1), (-1, 1, 1)]
    half = {19: half, 15: half[:3] + corners, 27: half + corners}[q]
    return np.array([(0, 0, 0)] + half + [tuple(-v for v in h) for h in half], dtype=np.int64)
