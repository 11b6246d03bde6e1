"""Three merged steps per pass (LBM_SWAP3, the deeper merging the paper's
conclusion names as its next step; the plain layout with one or two columns per thread,
FP32).  Every scheme runs the same per-cell arithmetic, so three merged steps
must equal three plain two-array steps to the bit: any difference is a race,
a missing halo cell or an indexing slip of the third level.  Covered: ragged
tiles, walls, a moving lid, a body force, remainders of one and two steps,
the three compiled tile shapes, rounds over bands of tile rows, the full 512^3
lattice against the two-step kernel, and the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import MOVING_WALL, PERIODIC, WALL, Oracle
from paper_2208_05429_amd import capi
from paper_2208_05429_amd import workloads as wl
from paper_2208_05429_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

NAMES = {PERIODIC: "periodic", WALL: "wall", MOVING_WALL: "moving"}
CASES = [
    ((20, 37, 45), (WALL, WALL, WALL, MOVING_WALL, WALL, WALL), (0.05, 0.0, -0.02)),
    ((23, 30, 61), (PERIODIC, PERIODIC, WALL, WALL, MOVING_WALL, WALL), (0.03, -0.02, 0.0)),
    ((17, 41, 33), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),
    ((26, 13, 70), (MOVING_WALL, WALL, PERIODIC, PERIODIC, WALL, WALL), (0.0, 0.04, 0.01)),
    ((19, 35, 130), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),
    ((9, 7, 5), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),  # one tile, a plane smaller than the halo frame
]


def _init(shape, seed):
    _, u0 = wl.taylor_green_3d(shape, 0.03)
    u0 = u0 + wl.uniform_noise(shape, 5e-3, seed)
    return torch.as_tensor(wl.random_density(shape, 0.01, seed + 1)), torch.as_tensor(u0)


def _agree(shape, faces, wall_u, steps_list, variant=0, force=None, seed=0):
    names = [NAMES[f] for f in faces]
    r0, u0 = _init(shape, seed)
    F = None if force is None else torch.as_tensor(force, dtype=torch.float32)
    ref = Lattice(shape, 0.6, "f32", "two_array", names, wall_u, F, rho0=r0, u0=u0)
    lat = Lattice(shape, 0.6, "f32", "swap3", names, wall_u, F, rho0=r0, u0=u0, variant=variant)
    for n in steps_list:
        print(f"[gpu] swap3 variant {variant} {shape} {names} {n} steps", flush=True)
        ref.step(n)
        lat.step(n)
        torch.cuda.synchronize()
        assert torch.equal(lat.f.view(torch.int32), ref.f.view(torch.int32)), (shape, variant, n)
    lat.close()
    ref.close()


@pytest.mark.parametrize("variant", [0, 1, 2])  # 16 x 32 with two columns per thread; 10 x 26, 16 x 16
@pytest.mark.parametrize("case", range(len(CASES)))
def test_three_merged_steps_equal_two_array_bitwise(case, variant):
    shape, faces, wall_u = CASES[case]
    _agree(shape, faces, wall_u, (3, 5, 7, 1), variant, seed=500 + case)  # remainders 0, 2, 1, 1


def test_three_merged_steps_with_a_body_force():
    shape = (24, 20, 18)
    faces = (PERIODIC, PERIODIC, WALL, WALL, WALL, WALL)
    _agree(shape, faces, (0, 0, 0), (6, 4), force=wl.normal_field(shape, 1e-4, 510), seed=511)
    _agree((18, 22, 40), (PERIODIC,) * 6, (0, 0, 0), (3, 2), variant=1, force=wl.normal_field((18, 22, 40), 1e-4, 512),
           seed=513)


@pytest.mark.parametrize("shape,faces,wall_u,variant", [
    ((6, 280, 290), (WALL, WALL, WALL, MOVING_WALL, WALL, WALL), (0.05, 0.0, 0.01), 1),  # 10 x 26: 28 x 12 tiles, 2 rounds
    ((5, 285, 266), (PERIODIC,) * 6, (0.0, 0.0, 0.0), 1),  # periodic y with a 5-row last tile row
    ((4, 512, 520), (WALL, WALL, PERIODIC, PERIODIC, WALL, WALL), (0.0, 0.0, 0.0), 2),  # 16 x 16 tiles across the seam
    # 16 x 32 tiles, two columns per thread: 17 x 32 tiles in bands of 8, 8 and 1 tile rows
    ((6, 272, 1024), (PERIODIC,) * 6, (0.0, 0.0, 0.0), 0),
])
def test_three_merged_steps_in_rounds_equal_two_array_bitwise(shape, faces, wall_u, variant):
    _agree(shape, faces, wall_u, (3, 4), variant=variant, seed=520)


def test_three_merged_steps_match_the_oracle():
    cfg = wl.TGV_32
    rho0, u0 = wl.taylor_green_3d(cfg["shape"], cfg["u0"])
    o = Oracle(cfg["shape"], cfg["tau"])
    ref = o.run(o.init(rho0, u0), cfg["steps"])
    rho_r, u_r, un_r = o.macro(ref)
    lat = Lattice(cfg["shape"], cfg["tau"], "f32", "swap3", rho0=torch.as_tensor(rho0), u0=torch.as_tensor(u0))
    lat.step(cfg["steps"])  # 33 three-step passes and one single step
    rho, u, un, _ = lat.macroscopic(sums=True)
    e = [float(np.abs(a.cpu().numpy() - b).max() / np.abs(b).max()) for a, b in ((rho, rho_r), (u, u_r), (un, un_r))]
    print(f"swap3 FP32 TGV 32^3 100 steps vs oracle: rho {e[0]:.2e} u {e[1]:.2e} |u| {e[2]:.2e}")
    assert max(e) <= 2e-6
    lat.close()


def test_three_merged_steps_at_512_cubed_equal_two_steps_bitwise():
    # the 512^3 Taylor-Green workload (16 x 32 tiles, two columns per thread,
    # in two rounds) against the two-step kernel of the bench, 6 steps each
    shape = (512, 512, 512)
    u0 = wl.taylor_green_3d_device(shape, 0.02, (0.0, 0.0, 0.0), "cuda")
    a = Lattice(shape, 0.6, "f32", "swap3", u0=u0)
    b = Lattice(shape, 0.6, "f32", "swap2", u0=u0)
    del u0
    print("[gpu] 512^3 swap3 vs swap2, 6 steps", flush=True)
    a.step(6)
    b.step(6)
    s = a.sums()
    torch.cuda.synchronize()
    assert torch.equal(a.f.view(torch.int32), b.f.view(torch.int32))
    assert np.isfinite(s).all()
    a.close()
    b.close()
