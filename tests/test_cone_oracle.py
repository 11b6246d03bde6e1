"""The neighbourhood construction the full-size GPU tests use to get exact
FP64 values of sampled cells: checked here on lattices small enough for the
oracle to run whole."""
import numpy as np
import pytest

from oracle import MOVING_WALL, PERIODIC, WALL, Oracle
from paper_2208_05429_amd import workloads as wl
from tests.test_gpu_fullsize import oracle_center


@pytest.mark.parametrize("faces,wall_u", [
    ((PERIODIC,) * 6, (0.0, 0.0, 0.0)),
    ((WALL, WALL, WALL, MOVING_WALL, WALL, WALL), (0.05, 0.0, 0.0)),
    ((PERIODIC, PERIODIC, WALL, WALL, MOVING_WALL, WALL), (0.03, -0.02, 0.0)),
])
def test_neighbourhood_run_reproduces_the_full_run(faces, wall_u):
    shape, tau, n = (18, 16, 20), 0.6, 4
    rho0, u0 = wl.taylor_green_3d(shape, 0.03)
    u0 = u0 + wl.uniform_noise(shape, 5e-3, 1)
    o = Oracle(shape, tau, faces=faces, wall_u=wall_u)
    full = o.run(o.init(rho0, u0), n)
    for c in [(0, 0, 0), (17, 15, 19), (9, 8, 10), (1, 15, 3), (5, 0, 19)]:
        got = oracle_center(rho0, u0, shape, faces, wall_u, tau, c, n)
        assert np.abs(got - full[(slice(None),) + c]).max() <= 1e-15, c


@pytest.mark.parametrize("q", [15, 27])
def test_neighbourhood_run_reproduces_the_full_run_of_the_other_sets(q):
    from oracle import OracleQ
    shape, tau, n = (14, 16, 12), 0.7, 3
    faces, wall_u = (PERIODIC, PERIODIC, WALL, MOVING_WALL, PERIODIC, PERIODIC), (0.04, 0.0, 0.01)
    rho0, u0 = wl.taylor_green_3d(shape, 0.03)
    u0 = u0 + wl.uniform_noise(shape, 5e-3, 2)
    o = OracleQ(shape, tau, q, faces=faces, wall_u=wall_u)
    full = o.run(o.init(rho0, u0), n)
    for c in [(0, 0, 0), (13, 15, 11), (7, 8, 6), (1, 15, 3), (5, 0, 11)]:
        got = oracle_center(rho0, u0, shape, faces, wall_u, tau, c, n, q=q)
        assert np.abs(got - full[(slice(None),) + c]).max() <= 1e-15, c
