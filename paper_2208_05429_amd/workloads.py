"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no lattice Boltzmann arithmetic: it only draws the initial
density/velocity fields and the body-force fields that both the CPU oracle and
the GPU library consume.  Every generator is deterministic in its seed.

Field layout: ``rho[x, y, z]`` and ``u[c, x, y, z]`` (SoA, z fastest), float64.
"""
from __future__ import annotations

import math

import numpy as np

# Workloads the library is exercised on (dims are nx x ny x nz, x slowest).
TGV_32 = dict(name="tgv32_fp64", shape=(32, 32, 32), tau=0.8, u0=0.02, steps=100)
CAVITY_256 = dict(name="cavity256_fp32", shape=(256, 256, 256), tau=0.52, lid_u=0.05, steps=1000)
TGV_512 = dict(name="tgv512_fp32", shape=(512, 512, 512), tau=0.6, u0=0.02, noise=1e-3, seed=20805429, steps=500)
CHANNEL_ADJ = dict(name="channel128x64x64_adjoint", shape=(128, 64, 64), tau=0.8, force_std=1e-6, force_seed=1,
                   target_seed=2, cell_seed=3, steps=200, checkpoint=20, fd_eps=1e-4, fd_cells=16)
TGV_1024 = dict(name="tgv1024_fp32", shape=(1024, 1024, 1024), tau=0.55, u0=0.02, phase_seed=4, steps=50)


def _grid(shape):
    return np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")


def taylor_green_3d(shape, u0, phase=(0.0, 0.0, 0.0)):
    """rho = 1 and u = (u0 sin X cos Y cos Z, -u0 cos X sin Y cos Z, 0) with
    X = k_x x + phase_x (k_a = 2 pi / n_a), evaluated on integer cell indices."""
    x, y, z = _grid(shape)
    X = 2 * math.pi * x / shape[0] + phase[0]
    Y = 2 * math.pi * y / shape[1] + phase[1]
    Z = 2 * math.pi * z / shape[2] + phase[2]
    u = np.empty((3,) + tuple(shape))
    u[0] = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    u[2] = 0.0
    return np.ones(shape), u


def taylor_green_2d(shape, u0, axes=(0, 1)):
    """Two-dimensional Taylor-Green vortex in the plane of ``axes``, constant
    along the third axis: u_a = u0 sin A cos B, u_b = -u0 cos A sin B."""
    a, b = axes
    g = _grid(shape)
    A = 2 * math.pi * g[a] / shape[a]
    B = 2 * math.pi * g[b] / shape[b]
    u = np.zeros((3,) + tuple(shape))
    u[a] = u0 * np.sin(A) * np.cos(B)
    u[b] = -u0 * np.cos(A) * np.sin(B)
    return np.ones(shape), u


def shear_wave(shape, amp, flow_axis=0, grad_axis=1):
    """u_flow = amp sin(2 pi y / n_y) along ``grad_axis``; rho = 1."""
    g = _grid(shape)
    u = np.zeros((3,) + tuple(shape))
    u[flow_axis] = amp * np.sin(2 * math.pi * g[grad_axis] / shape[grad_axis])
    return np.ones(shape), u


def uniform_noise(shape, amp, seed, comps=3):
    """i.i.d. U[-amp, amp] per component per cell (numpy default_rng(seed))."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(comps,) + tuple(shape))


def normal_field(shape, std, seed, comps=3):
    """i.i.d. N(0, std^2) per component per cell (numpy default_rng(seed))."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, std, size=(comps,) + tuple(shape))


def random_density(shape, amp, seed):
    """rho = 1 + U[-amp, amp] per cell."""
    rng = np.random.default_rng(seed)
    return 1.0 + rng.uniform(-amp, amp, size=tuple(shape))


def tgv_512_fields(shape=None, u0=None, noise=None, seed=None):
    """The 512^3 workload's initial fields: 3D Taylor-Green plus seeded noise."""
    cfg = TGV_512
    shape = shape or cfg["shape"]
    rho, u = taylor_green_3d(shape, u0 if u0 is not None else cfg["u0"])
    u += uniform_noise(shape, noise if noise is not None else cfg["noise"], seed if seed is not None else cfg["seed"])
    return rho, u


def random_phases(seed):
    """Three phases ~ U[0, 2 pi) for the random-phase Taylor-Green field."""
    rng = np.random.default_rng(seed)
    return tuple(float(p) for p in rng.uniform(0.0, 2 * math.pi, size=3))


def taylor_green_3d_at(shape, u0, phase, ix, iy, iz):
    """The Taylor-Green field of taylor_green_3d on the index grid ix x iy x iz
    (1-D integer arrays): u of shape (3, len(ix), len(iy), len(iz))."""
    X = (2 * math.pi * np.asarray(ix, np.float64) / shape[0] + phase[0])[:, None, None]
    Y = (2 * math.pi * np.asarray(iy, np.float64) / shape[1] + phase[1])[None, :, None]
    Z = (2 * math.pi * np.asarray(iz, np.float64) / shape[2] + phase[2])[None, None, :]
    u = np.zeros((3, len(ix), len(iy), len(iz)))
    u[0] = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    return u


def taylor_green_3d_device(shape, u0, phase, device):
    """The same field built directly in device memory (float64 torch tensor of
    shape (3, nx, ny, nz)), for lattices whose fields are too large for the
    host.  Same formula as taylor_green_3d_at, evaluated by torch."""
    import torch
    ax = [(2 * math.pi * torch.arange(n, dtype=torch.float64, device=device)) / n + p for n, p in zip(shape, phase)]
    sx, cx = torch.sin(ax[0])[:, None, None], torch.cos(ax[0])[:, None, None]
    sy, cy = torch.sin(ax[1])[None, :, None], torch.cos(ax[1])[None, :, None]
    cz = torch.cos(ax[2])[None, None, :]
    u = torch.zeros((3,) + tuple(shape), dtype=torch.float64, device=device)
    u[0] = ((u0 * sx) * cy) * cz
    u[1] = ((-u0 * cx) * sy) * cz
    return u


def sample_cells(shape, count, seed):
    """``count`` distinct cell indices (x, y, z) drawn with default_rng(seed)."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(int(np.prod(shape)), size=count, replace=False)
    return [tuple(int(v) for v in np.unravel_index(i, shape)) for i in flat]
