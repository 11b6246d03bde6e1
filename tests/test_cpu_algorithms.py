"""The paper's sequential CPU algorithms (liblbm_cpu.so, include/lbm_cpu.h):
Fuse Swap (Sec. 3, Alg. 1) and the two-step memory-aware sweep with prism
traversal (Sec. 4.1, Alg. 2).  Sec. 5.1 verifies the paper's algorithms by
their giving the same result as the plain solvers; here they are held to the
FP64 oracle (plain two-array collide + stream), the two-step schedule is
checked cell by cell for the states the swap algorithm requires of every
partner (checked mode), and the two algorithms agree to the bit (each cell
collides the same values whatever the order of the swaps)."""
import numpy as np
import pytest

from oracle import MOVING_WALL, PERIODIC, WALL, Oracle
from paper_2208_05429_amd import capi, host
from paper_2208_05429_amd import workloads as wl

LID = (WALL, WALL, WALL, MOVING_WALL, WALL, WALL)
WALLS = (WALL,) * 6


def _start(shape, tau, faces, wall_u, seed=3, amp=0.03):
    rho0 = wl.random_density(shape, 0.02, seed)
    _, u0 = wl.taylor_green_3d(shape, amp)
    u0 = u0 + wl.uniform_noise(shape, 5e-3, seed + 1)
    cfg = capi.make_config(shape, tau, faces=faces, wall_u=wall_u)
    o = Oracle(shape, tau, faces=faces, wall_u=wall_u)
    return cfg, o, o.init(rho0, u0), host.lbm_cpu_init(cfg, rho0, u0)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_init_is_the_oracle_equilibrium():
    cfg, o, f0, g = _start((5, 6, 7), 0.7, LID, (0.05, 0, 0))
    assert _rel(host.to_soa_f(g), f0) <= 1e-15


@pytest.mark.parametrize("shape,faces", [
    ((5, 6, 7), LID),
    ((4, 4, 4), WALLS),
    ((6, 5, 4), (PERIODIC,) * 6),
    ((7, 4, 6), (PERIODIC, PERIODIC, WALL, MOVING_WALL, WALL, WALL)),
    ((3, 8, 5), (WALL, WALL, PERIODIC, PERIODIC, MOVING_WALL, WALL)),
    ((2, 3, 2), (PERIODIC,) * 6),
])
def test_fuse_swap_matches_the_oracle(shape, faces):
    wall_u = (0.05, 0.0, 0.0) if MOVING_WALL in faces[:4] else (0.0, 0.04, 0.0)
    cfg, o, f0, g = _start(shape, 0.7, faces, wall_u)
    f = f0
    for n in (1, 2, 3):
        host.lbm_cpu_fuse_swap(cfg, g, n)
        f = o.run(f, n)
        assert _rel(host.to_soa_f(g), f) <= 1e-14, (shape, n)


@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 6, 7), (8, 9, 10), (3, 3, 3), (6, 2, 5), (5, 7, 2), (1, 4, 5),
                                   (4, 1, 3), (2, 2, 2), (9, 5, 12)])
@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 7])
def test_two_step_schedule_and_result(shape, tile):
    # lid-driven cavity (every face a wall, the +y lid moving along x): the
    # schedule is verified before every computation, the result against the
    # oracle, and against Fuse Swap to the bit, over even and odd step counts
    cfg, o, f0, g = _start(shape, 0.7, LID, (0.05, 0.0, 0.0))
    g_fs = g.copy()
    f = f0
    for n in (2, 5):
        host.lbm_cpu_two_step(cfg, g, n, tile=tile, checked=True)
        host.lbm_cpu_fuse_swap(cfg, g_fs, n)
        f = o.run(f, n)
        assert np.array_equal(g, g_fs), (shape, tile, n)
        assert _rel(host.to_soa_f(g), f) <= 1e-14, (shape, tile, n)


def test_two_step_paper_example_cube_with_prisms():
    # the 4x4x4 cube of Sec. 4.1 (Fig. 2) and the 4x16x16 cuboid swept with
    # stride 4 (Fig. 3)
    for shape in ((4, 4, 4), (4, 16, 16)):
        cfg, o, f0, g = _start(shape, 0.6, LID, (0.05, 0.0, 0.0))
        host.lbm_cpu_two_step(cfg, g, 4, tile=4, checked=True)
        assert _rel(host.to_soa_f(g), o.run(f0, 4)) <= 1e-14


def test_unsupported_and_invalid():
    g = np.zeros((4, 4, 4, 19))
    with pytest.raises(capi.LbmError) as e:
        host.lbm_cpu_two_step(capi.make_config((4, 4, 4), 0.7), g, 2)  # periodic
    assert e.value.status == capi.LBM_EUNSUPPORTED
    with pytest.raises(capi.LbmError) as e:
        host.lbm_cpu_fuse_swap(capi.make_config((4, 4, 4), 0.7, use_force=True), g, 1)
    assert e.value.status == capi.LBM_EUNSUPPORTED
    with pytest.raises(capi.LbmError) as e:
        host.lbm_cpu_fuse_swap(capi.make_config((4, 4, 4), 0.5), g, 1)
    assert e.value.status == capi.LBM_EINVAL


def test_cpu_library_exports_its_header():
    import re
    L = host.lib()
    names = set(re.findall(r"^\s*lbm_status\s+(lbm_cpu_\w+)\s*\(", open(host.HEADER).read(), re.M))
    assert names == {"lbm_cpu_init", "lbm_cpu_fuse_swap", "lbm_cpu_two_step"}
    for n in names:
        assert hasattr(L, n)
