"""GPU parity at the full workload sizes, in the launch configuration the bench
times, on sampled cells.

After n steps a cell depends only on the initial cells within Chebyshev
distance n (a D3Q19 population moves at most one cell per axis per step).
For each sampled cell the FP64 oracle runs on the (2n+3)^3 neighbourhood of
the initial field: periodic axes are wrapped into the box; where the box
meets a wall of the domain it is cut there and the wall kept, and every other
box face is an artificial wall at least n+1 cells away, outside the cone.  The
centre of that small run is the exact FP64 answer for the sampled cell.
"""
import numpy as np
import pytest
import torch

from oracle import MOVING_WALL, PERIODIC, WALL, Oracle
from paper_2208_05429_amd import workloads as wl
from paper_2208_05429_amd.lattice import Lattice

pytestmark = pytest.mark.gpu


def cone_box(shape, faces, center, n):
    """Index arrays of the neighbourhood box and the oracle faces for it."""
    R = n + 1
    idx, box_faces, pos = [], [], []
    for a in range(3):
        c, L = center[a], shape[a]
        if faces[2 * a] == PERIODIC:
            idx.append(np.arange(c - R, c + R + 1) % L)
            box_faces += [WALL, WALL]
            pos.append(R)
        else:
            lo, hi = max(0, c - R), min(L, c + R + 1)
            idx.append(np.arange(lo, hi))
            box_faces += [faces[2 * a] if lo == 0 else WALL, faces[2 * a + 1] if hi == L else WALL]
            pos.append(c - lo)
    return idx, tuple(box_faces), tuple(pos)


def oracle_center(rho0, u0, shape, faces, wall_u, tau, center, n):
    idx, bfaces, pos = cone_box(shape, faces, center, n)
    ix = np.ix_(*idx)
    r = None if rho0 is None else np.ascontiguousarray(rho0[ix])
    u = None if u0 is None else np.ascontiguousarray(np.stack([u0[c][ix] for c in range(3)]))
    bshape = tuple(len(i) for i in idx)
    o = Oracle(bshape, tau, faces=bfaces, wall_u=wall_u)
    f = o.run(o.init(r, u), n)
    return f[(slice(None),) + pos]


def gpu_cells(lat, cells):
    f = lat.f
    out = []
    for c in cells:
        out.append(f[(slice(None),) + tuple(c)].to(torch.float64).cpu().numpy())
    from paper_2208_05429_amd.lattice import lattice_weights
    return np.array(out) + lattice_weights()[None, :]


def test_tgv512_fp32_merged_sampled_cells():
    cfg = wl.TGV_512
    shape, tau, n = cfg["shape"], cfg["tau"], 4
    print(f"[gpu] 512^3 f32 swap2 sampled cells, {n} steps", flush=True)
    _, u0 = wl.tgv_512_fields(shape)
    lat = Lattice(shape, tau, "f32", "swap2", u0=torch.from_numpy(u0))
    s0 = lat.sums()
    lat.step(n)
    torch.cuda.synchronize()
    s1 = lat.sums()
    cells = wl.sample_cells(shape, 16, 7) + [(0, 0, 0), (511, 511, 511), (0, 511, 0), (256, 0, 511)]
    got = gpu_cells(lat, cells)
    faces = (PERIODIC,) * 6
    for c, g in zip(cells, got):
        ref = oracle_center(None, u0, shape, faces, (0, 0, 0), tau, c, n)
        assert np.abs(g - ref).max() <= 2e-7, c  # FP32 rounding of values <= 1/3 over a few steps
    # exact invariants of the update, at the full size: mass and momentum
    assert abs(s1[0] - s0[0]) <= 1e-9 * s0[0]
    assert np.abs(s1[1:] - s0[1:]).max() <= 1e-9 * s0[0]
    lat.close()
    del lat
    torch.cuda.empty_cache()


@pytest.mark.parametrize("scheme", ["swap2", "swap1", "two_array"])
def test_cavity256_fp32_sampled_cells(scheme):
    cfg = wl.CAVITY_256
    shape, tau, n = cfg["shape"], cfg["tau"], 6
    faces = (WALL, WALL, WALL, MOVING_WALL, WALL, WALL)
    wall_u = (cfg["lid_u"], 0.0, 0.0)
    print(f"[gpu] 256^3 cavity f32 {scheme} sampled cells, {n} steps", flush=True)
    lat = Lattice(shape, tau, "f32", scheme, ["wall", "wall", "wall", "moving", "wall", "wall"], wall_u)
    lat.step(n)
    torch.cuda.synchronize()
    L = shape[0]
    cells = [(0, L - 1, 0), (L - 1, L - 1, L - 1), (L // 2, L - 1, L // 2), (3, L - 2, 100), (L - 1, L - 3, 0),
             (0, 0, 0), (128, 128, 128), (200, L - 1, 5), (17, L - 4, L - 2)]
    got = gpu_cells(lat, cells)
    for c, g in zip(cells, got):
        ref = oracle_center(None, None, shape, faces, wall_u, tau, c, n)
        assert np.abs(g - ref).max() <= 2e-7, c
    lat.close()
